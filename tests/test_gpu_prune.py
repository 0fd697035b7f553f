"""Locality-pruned passes (prune_u > 0) against the exact FP64 oracle.  With
prune_u = 30 every skipped term is below exp(-30) ~ 1e-13, far under the FP32
rounding of R, so the bar is the exact path's: identical track sets after
matching, parameters within 1e-4 relative, R within 1e-5; and the pruned GPU
path lands within 1e-6 of the unpruned GPU path seed by seed for at least 95%
of the seeds converged on both (the hits of a plane are visited in sorted
order, so FP32 sums round differently and a seed on a basin boundary may go
the other way, as between the GPU and the oracle)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events, retina

from gpu_util import assert_tracks_match, event_tracks

pytestmark = pytest.mark.gpu
U = 30.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


def _find(ctx, b, P, **kw):
    return ctx.retina_find_tracks(b.meas_dim, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P, **kw)


def _check(ctx, b, P, z0, z1, seeds=None, offs=None):
    kw = {} if seeds is None else dict(seeds=seeds, seed_offsets=offs)
    res = _find(ctx, b, dict(P, prune_u=U), want_seeds=True, **kw)
    ref = oracle.find_tracks(b, P, **kw)
    for e in range(b.n_events):
        th, R = event_tracks(res, e, b.meas_dim)
        a, c = ref["track_offsets"][e], ref["track_offsets"][e + 1]
        err = assert_tracks_match(b.meas_dim, th, R, ref["theta"][a:c], ref["R"][a:c], P["d_merge"], z0, z1)
        _say("  event %d: %d tracks, max parameter error %.2e" % (e, len(R), err.max() if len(err) else 0.0))
    exact = _find(ctx, b, P, want_seeds=True, **kw)
    d = np.abs(res["seed_theta"] - exact["seed_theta"]).max(axis=1)
    both = (res["seed_flags"] & 1).astype(bool) & (exact["seed_flags"] & 1).astype(bool)
    assert np.mean(d[both] < 1e-6) >= 0.95
    return res


def test_prune_c2_lattice(ctx):
    _say("pruned: c2 event, 64 x 64 lattice")
    cfg = events.load_config("c2")
    _check(ctx, events.make_batch(cfg), cfg["params"], 20.0, 750.0)


def test_prune_c3_events_explicit_seeds(ctx):
    _say("pruned: c3 events 0..3, seeds near the tracks plus random ones")
    cfg = events.load_config("c3")
    b = events.make_batch(cfg, 4)
    rng = np.random.default_rng(2)
    seeds, offs = [], [0]
    for e in range(4):
        t = b.truth[e]
        s = np.zeros((len(t) + 64, 4))
        s[: len(t), 2:] = t[:, 2:] + rng.normal(0, 0.002, (len(t), 2))
        s[len(t):, 2:] = rng.uniform(-0.3, 0.3, (64, 2))
        seeds.append(s.astype(np.float32).astype(np.float64))
        offs.append(offs[-1] + len(s))
    _check(ctx, b, cfg["params"], 20.0, 750.0, np.concatenate(seeds), np.array(offs, np.int64))


def test_prune_c1_meas_dim_one(ctx):
    _say("pruned: c1 (meas_dim 1)")
    cfg = events.load_config("c1")
    for idx in range(3):
        _check(ctx, events.make_batch(cfg, 1, start=idx), cfg["params"], 1.0, 8.0)


def test_prune_svelo_origin_constrained(ctx):
    _say("pruned: simplified VELO, prior seeds, offsets held")
    cfg = events.load_config("c8")
    zp = events.plane_z(cfg)
    b = events.batch_from_events(2, zp, [events.make_event(cfg, i, zp) for i in (0, 1)])
    s, o = events.prior_seeds(cfg, 1024, [0, 1])
    _check(ctx, b, cfg["params"], float(zp[0]), float(zp[-1]), s, o)


def test_prune_tiled_events(ctx):
    """An event streamed through a 1024-hit tile: each tile's part of a plane is
    still sorted, and pruning works per tile."""
    _say("pruned: c2 event through a 1024-hit tile")
    cfg = events.load_config("c2")
    b = events.make_batch(cfg)
    old = ctx.retina_get_tuning(2, 0)
    try:
        ctx.retina_set_tuning(2, 0, 1, 1024)
        _check(ctx, b, dict(cfg["params"], lattice_n=[32, 32]), 20.0, 750.0)
    finally:
        ctx.retina_set_tuning(2, 0, old["cand"], old["tile_hits"])


def test_prune_runs_are_bit_identical(ctx):
    """The pruned passes visit the hit window of the points a wave holds, so
    the line search must put its pending points into waves in the same order on
    every run: repeated calls (lattice through a 1024-hit tile, one candidate
    per lane with several lanes per seed; and the learned-seeding shape on c3
    events) give the same bits."""
    _say("pruned: repeated calls are bit-identical")
    cfg = events.load_config("c2")
    b = events.make_batch(cfg)
    P = dict(cfg["params"], lattice_n=[32, 32], prune_u=U)
    old = ctx.retina_get_tuning(2, 0)
    try:
        ctx.retina_set_tuning(2, 0, 1, 1024)
        runs = [_find(ctx, b, P, want_seeds=True) for _ in range(3)]
    finally:
        ctx.retina_set_tuning(2, 0, old["cand"], old["tile_hits"])
    for r in runs[1:]:
        for k in ("seed_theta", "seed_R", "seed_flags", "seed_nreval", "track_offsets"):
            assert r[k].tobytes() == runs[0][k].tobytes(), k
        assert r["tracks"].tobytes() == runs[0]["tracks"].tobytes()
    c3 = events.load_config("c3")
    b3 = events.make_batch(c3, 4)
    rng = np.random.default_rng(5)
    seeds, offs = [], [0]
    for e in range(4):
        t = b3.truth[e]
        s = np.zeros((len(t), 4))
        s[:, 2:] = t[:, 2:] + rng.normal(0, 0.002, (len(t), 2))
        seeds.append(s.astype(np.float32).astype(np.float64))
        offs.append(offs[-1] + len(s))
    S, O = np.concatenate(seeds), np.array(offs, np.int64)
    runs = [_find(ctx, b3, dict(c3["params"], prune_u=U), seeds=S, seed_offsets=O, want_seeds=True)
            for _ in range(3)]
    for r in runs[1:]:
        assert r["seed_theta"].tobytes() == runs[0]["seed_theta"].tobytes()
        assert r["tracks"].tobytes() == runs[0]["tracks"].tobytes()


def test_prune_long_plane_stays_exact(ctx):
    """A plane with more than 4096 hits cannot be sorted in LDS: that event runs
    unpruned (same results as prune_u = 0 within rounding) while the others of
    the batch are pruned."""
    _say("pruned: an event with 5000 hits on one plane")
    cfg = events.load_config("c2")
    zp = events.plane_z(cfg)
    ev = events.make_event(cfg, 0, zp)
    rng = np.random.default_rng(4)
    extra = 5000
    x = np.concatenate([ev.x, rng.uniform(-40, 40, extra).astype(np.float32)])
    y = np.concatenate([ev.y, rng.uniform(-40, 40, extra).astype(np.float32)])
    pl = np.concatenate([ev.plane, np.full(extra, 3, np.int32)])
    big = events.Event(x, y, pl, np.concatenate([ev.label, np.full(extra, -1, np.int32)]), ev.truth, ev.truth_nhits)
    b = events.batch_from_events(2, zp, [big, events.make_event(cfg, 0, zp)])
    P = dict(cfg["params"], lattice_n=[32, 32])
    res = _find(ctx, b, dict(P, prune_u=U))
    exact = _find(ctx, b, P)
    for e in range(2):
        th, R = event_tracks(res, e, 2)
        th0, R0 = event_tracks(exact, e, 2)
        assert_tracks_match(2, th, R, th0, R0, P["d_merge"], 20.0, 750.0)


def test_prune_arguments(ctx):
    cfg = events.load_config("c2")
    b = events.make_batch(cfg)
    for bad in (dict(cfg["params"], prune_u=-1.0), dict(cfg["params"], prune_u=float("nan")),
                dict(cfg["params"], prune_u=30.0, update="bfgs")):
        with pytest.raises(retina.RetinaError) as ei:
            _find(ctx, b, bad)
        assert ei.value.code == retina.ERR_INVALID_ARG
