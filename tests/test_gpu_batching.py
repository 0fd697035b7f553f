"""Batching row: one captured HIP graph serves batches of different shapes,
replays equal eager launches bit for bit, and the autotuner picks a valid
launch shape whose results keep parity."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events, retina

from gpu_util import assert_tracks_match, event_tracks

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


def _find(ctx, b, P, **kw):
    return ctx.retina_find_tracks(b.meas_dim, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P, **kw)


def test_graph_replays_equal_eager(ctx):
    cfg = events.load_config("c3")
    P = cfg["params"]
    batches = [events.make_batch(cfg, n, start=s) for n, s in ((5, 0), (12, 40), (1, 7), (5, 0))]
    ctx.retina_set_graphs(False)
    eager = [_find(ctx, b, P) for b in batches]
    ctx.retina_set_graphs(True)
    for rep in range(3):
        _say("graph replay round %d" % rep)
        for b, ref in zip(batches, eager):
            got = _find(ctx, b, P)
            np.testing.assert_array_equal(got["tracks"], ref["tracks"])
            np.testing.assert_array_equal(got["track_offsets"], ref["track_offsets"])
            # eager work between replays (a response call uses the same context and pool)
            ctx.retina_response(2, b.plane_z, b.event_offsets[:2], b.x[:b.event_offsets[1]],
                                b.y[:b.event_offsets[1]], b.plane[:b.event_offsets[1]],
                                np.zeros((3, 4), np.float32), sigma=1.0)


def test_profiling_leaves_no_hip_error_behind(ctx):
    """Regression: profiled calls with graphs enabled must not leave a pending HIP
    error that a later torch launch check or library call would report."""
    import torch
    cfg = events.load_config("c3")
    b = events.make_batch(cfg, 3)
    ctx.retina_set_graphs(True)
    ctx.retina_set_profiling(True)
    ctx.retina_profile_reset()
    for _ in range(2):
        _find(ctx, b, cfg["params"])
    prof = ctx.retina_get_profile()
    ctx.retina_set_profiling(False)
    assert prof["calls"] == 2 and prof["ms_hot"] > 0 and prof["exec_pairs"] > 0
    t = torch.zeros(1000, device="cuda")
    torch.cuda.synchronize()
    assert float(t.sum()) == 0.0
    _find(ctx, b, cfg["params"])


def test_autotune_installs_valid_shape_and_keeps_parity(ctx, tmp_path):
    cfg = events.load_config("c3")
    P = cfg["params"]
    sample = events.make_batch(cfg, 16, start=100)
    cache = str(tmp_path / "tune.txt")
    _say("autotune")
    choice = ctx.retina_autotune(2, sample.plane_z, sample.event_offsets, sample.x, sample.y, sample.plane,
                                 P, cache_path=cache)
    assert choice["cand"] in (1, 2) and 2048 <= choice["tile_hits"] <= 12288
    assert ctx.retina_get_tuning(2, 0)["cand"] == choice["cand"]
    txt = open(cache).read()
    assert "meas_dim=2" in txt and ("cand=%d tile=%d" % (choice["cand"], choice["tile_hits"])) in txt
    # second call reuses the cache (no new line)
    again = ctx.retina_autotune(2, sample.plane_z, sample.event_offsets, sample.x, sample.y, sample.plane,
                                P, cache_path=cache)
    assert again == choice and open(cache).read() == txt
    b = events.make_batch(cfg, 2, start=300)
    res = _find(ctx, b, P)
    ref = oracle.find_tracks(b, P)
    for e in range(2):
        th, R = event_tracks(res, e, 2)
        a, c = ref["track_offsets"][e], ref["track_offsets"][e + 1]
        assert_tracks_match(2, th, R, ref["theta"][a:c], ref["R"][a:c], P["d_merge"], 20.0, 750.0)


def test_sparse_seeding_has_its_own_tuned_shape(ctx, tmp_path):
    """A batch with few explicit seeds per event (as from the proposer) is timed
    and installed in the sparse-seeding slot (kernel 2); the lattice slot stays."""
    cfg = events.load_config("c3")
    P = cfg["params"]
    sample = events.make_batch(cfg, 16, start=200)
    seeds, offs = [], [0]
    for e in range(sample.n_events):
        t = sample.truth[e].copy()
        t[:, :2] = 0.0
        seeds.append(np.round(t, 2))
        offs.append(offs[-1] + len(t))
    seeds = np.concatenate(seeds)
    offs = np.array(offs, np.int64)
    assert offs[-1] < 512 * sample.n_events
    dense = ctx.retina_get_tuning(2, 0)
    _say("autotune sparse")
    choice = ctx.retina_autotune(2, sample.plane_z, sample.event_offsets, sample.x, sample.y, sample.plane,
                                 P, cache_path=str(tmp_path / "tune.txt"), seeds=seeds, seed_offsets=offs)
    got = ctx.retina_get_tuning(2, 2)
    assert (got["cand"], got["tile_hits"]) == (choice["cand"], choice["tile_hits"])
    assert ctx.retina_get_tuning(2, 0) == dense
    res = _find(ctx, sample, P, seeds=seeds, seed_offsets=offs)
    ref = oracle.find_tracks(sample, P, seeds=seeds, seed_offsets=offs)
    for e in range(3):
        th, R = event_tracks(res, e, 2)
        a, c = ref["track_offsets"][e], ref["track_offsets"][e + 1]
        assert_tracks_match(2, th, R, ref["theta"][a:c], ref["R"][a:c], P["d_merge"], 20.0, 750.0)


def test_learned_step_graph_equals_eager_and_explicit_seeds(ctx):
    """The learned entry point runs proposer, ascent and merge as one device
    sequence (one captured graph).  Its replays, across batches of different
    shapes (each a new capture) and with eager library work in between, equal
    its eager launches bit for bit and equal the two-call path: the proposer's
    seeds read back and passed to retina_find_tracks as explicit seeds."""
    import torch
    from paper_1709_08610_amd import learned
    cfg = events.load_config("c3")
    LS = learned.settings(cfg)
    PL = LS["params"]
    model = ctx.retina_model_load(LS["model"])
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    batches = [events.make_batch(cfg, n, start=s) for n, s in ((6, 0), (17, 30), (6, 0))]

    def learned_call(b):
        d = (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))
        r = ctx.retina_find_tracks_learned(model, b.plane_z, *d, PL, LS["k_max"], LS["tau"], LS["conf_min"],
                                           nms=LS["nms"])
        torch.cuda.synchronize()
        return (retina.tracks_from_device(r), r["track_offsets"].cpu().numpy(), r["event_flags"].cpu().numpy())

    ctx.retina_set_graphs(False)
    eager = [learned_call(b) for b in batches]
    ctx.retina_set_graphs(True)
    for rep in range(3):
        _say("learned graph round %d" % rep)
        for b, (tr, toff, fl) in zip(batches, eager):
            gtr, gtoff, gfl = learned_call(b)
            np.testing.assert_array_equal(gtoff, toff)
            np.testing.assert_array_equal(gtr, tr)
            np.testing.assert_array_equal(gfl, fl)
            ctx.retina_response(2, b.plane_z, b.event_offsets[:2], b.x[:b.event_offsets[1]],
                                b.y[:b.event_offsets[1]], b.plane[:b.event_offsets[1]],
                                np.zeros((3, 4), np.float32), sigma=1.0)
    # the two-call path on the same seeds
    for b, (tr, toff, fl) in zip(batches[:2], eager[:2]):
        prop = ctx.retina_propose_seeds(model, b.plane_z, b.event_offsets, b.x, b.y, b.plane, LS["k_max"], LS["tau"],
                                        LS["conf_min"], PL, nms=LS["nms"])
        res = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, PL, seeds=prop["seeds"],
                                     seed_offsets=prop["seed_offsets"])
        np.testing.assert_array_equal(res["track_offsets"], toff)
        np.testing.assert_array_equal(res["tracks"], tr)
        np.testing.assert_array_equal(fl & 16, np.where(prop["fallback"] != 0, 16, 0))
