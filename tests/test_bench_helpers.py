"""bench.py's FP32-vs-FP64 comparison of track sets (the report beside the
CPU baseline), on oracle results: identical inputs give zero errors and no
one-sided tracks; FP32 rounding of the oracle's own values gives errors of
FP32 size; a dropped or an added track is counted on the right side."""
import numpy as np

import bench
import oracle
from paper_1709_08610_amd import events


def _ref():
    cfg = events.load_config("c1")
    b = events.make_batch(cfg, 3)
    return cfg, oracle.find_tracks(b, cfg["params"])


def test_identical_track_sets():
    cfg, ref = _ref()
    r = bench.fp32_vs_fp64(1, ref["theta"], ref["R"], ref["track_offsets"], ref, cfg["params"]["d_merge"], 1.0, 8.0)
    n = int(ref["track_offsets"][-1])
    assert r == dict(events=3, matched_tracks=n, gpu_only=0, oracle_only=0, max_rel_dtheta=0.0, max_rel_dR=0.0)


def test_rounding_and_one_sided_tracks():
    cfg, ref = _ref()
    th = ref["theta"].astype(np.float32).astype(np.float64)
    R = ref["R"].astype(np.float32)
    toff = ref["track_offsets"].copy()
    n = int(toff[-1])
    # event 0 loses its first track; event 2 gains a line far from every track
    th = np.delete(th, 0, axis=0)
    R = np.delete(R, 0)
    toff[1:] -= 1
    th = np.vstack([th, [[0.49, -0.99]]])
    R = np.append(R, 3.0)
    toff[3] += 1
    r = bench.fp32_vs_fp64(1, th, R, toff, ref, cfg["params"]["d_merge"], 1.0, 8.0)
    assert r["matched_tracks"] == n - 1 and r["oracle_only"] == 1 and r["gpu_only"] == 1
    assert 0.0 < r["max_rel_dtheta"] < 2.0 ** -23
    assert 0.0 < r["max_rel_dR"] < 2.0 ** -23
