"""GPU parity on the simplified VELO of Section 3: tracks from the origin,
seeds drawn from the track prior, the ascent and the FP64 polish on the slope
block only (offsets held at 0).  Same bar as the other track-set parity tests:
identical track sets after matching within d_merge, parameters within 1e-4
relative (scale floors), R within 1e-5."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events, retina

from gpu_util import assert_tracks_match, event_tracks

pytestmark = pytest.mark.gpu


def test_svelo_find_tracks_parity():
    print("svelo: 3 events x 200 tracks, 2048 prior seeds each", flush=True)
    sys.stdout.flush()
    ctx = retina.Context(0)
    cfg = events.load_config("c8")
    P = cfg["params"]
    zp = events.plane_z(cfg)
    idx = [0, 1, 2]
    b = events.batch_from_events(2, zp, [events.make_event(cfg, i, zp) for i in idx])
    seeds, offs = events.prior_seeds(cfg, 2048, idx)
    res = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P, seeds=seeds,
                                 seed_offsets=offs, want_seeds=True)
    ref = oracle.find_tracks(b, P, seeds=seeds, seed_offsets=offs)
    assert np.all(res["seed_theta"][:, :2] == 0.0), "offsets moved"
    z0, z1 = float(zp[0]), float(zp[-1])
    for e in range(3):
        th, R = event_tracks(res, e, 2)
        a, c = ref["track_offsets"][e], ref["track_offsets"][e + 1]
        err = assert_tracks_match(2, th, R, ref["theta"][a:c], ref["R"][a:c], P["d_merge"], z0, z1)
        print("  event %d: %d tracks, max parameter error %.2e" % (e, len(R), err.max() if len(err) else 0.0),
              flush=True)
    conv = (res["seed_flags"] & 1).astype(bool) & (ref["seed_flags"] & 1).astype(bool)
    d = np.abs(res["seed_theta"] - ref["seed_theta"]).max(axis=1)
    assert np.mean(d[conv] < 1e-6) > 0.97
