"""The grid-search vs multi-start comparison of Section 3 (Fig. 3) on the GPU:
with seeds costing a third of the grid search (counted with the measured T0,
C0 and q), the multi-start finds as many tracks by the paper's 1e-3 criterion
as the grid search does, at the lowest and highest track counts of the scan.
And the cost ratio C of the paper's footnote to Section 2 (one evaluation of
R with its gradient and Hessian against one of R alone), measured on a batch
that fills the GPU: above 1, and below the paper's 3 (the sums are factored
per plane, so the derivatives add six running sums to one exp per pair)."""
import sys

import pytest

from paper_1709_08610_amd import budget, events, retina

pytestmark = pytest.mark.gpu


def test_multistart_at_a_third_of_the_grid_cost():
    print("alpha budget: c7 scan, 50 and 350 tracks, 256 events each", flush=True)
    sys.stdout.flush()
    ctx = retina.Context(0)
    cfg = events.load_config("c7")
    out = budget.run(ctx, cfg, counts=[50, 350], events_per_point=256, reps=2,
                     log=lambda m: print(m, flush=True))
    P = cfg["params"]
    assert out["q"] == len(P["sigma"]) + P["n_final_steps"] + P["n_polish"] and out["C0"] > 0
    for row in out["points"]:
        g, a3, a10 = row["grid"], row["alpha_0.3333"], row["alpha_0.1"]
        assert g["eff_eps"] >= 0.9
        assert a3["eff_eps"] >= 0.95 and a3["eff_eps"] >= g["eff_eps"] - 0.02
        assert a3["cost_ratio"] <= 0.6          # a third by construction; timing noise allowed
        assert a10["seeds"] < a3["seeds"]
        assert a3["fake_rate"] <= 0.02


def test_multistart_budget_on_the_simplified_velo():
    """The same comparison on the paper's own workload (simplified VELO, seeds
    drawn from the track prior, 1e-3 rad between directions): at a third of the
    grid's cost the multi-start finds at least 90% of the tracks and about as many
    as the grid search; at a tenth it loses efficiency as the tracks get dense."""
    print("alpha budget: c8 scan, 50 and 350 tracks, 256 events each", flush=True)
    sys.stdout.flush()
    ctx = retina.Context(0)
    out = budget.run(ctx, events.load_config("c8"), counts=[50, 350], events_per_point=256, reps=2,
                     log=lambda m: print(m, flush=True))
    rows = out["points"]
    for row in rows:
        g, a3 = row["grid"], row["alpha_0.3333"]
        assert a3["eff_angle"] >= 0.9 and a3["eff_angle"] >= g["eff_angle"] - 0.03
        assert a3["cost_ratio"] <= 0.6
    assert rows[1]["alpha_0.1"]["eff_angle"] < rows[0]["alpha_0.1"]["eff_angle"] - 0.05


def test_cost_ratio_of_derivatives():
    import numpy as np
    import torch
    print("cost ratio C: 256 c3 events x 1024 lattice lines, R only and R + grad + Hess", flush=True)
    sys.stdout.flush()
    ctx = retina.Context(0)
    cfg = events.load_config("c3")
    b = events.make_batch(cfg, 256)
    n = 32
    v = -0.25 + (np.arange(n) + 0.5) * 0.5 / n
    th = np.zeros((n * n, 4), np.float32)
    th[:, 2] = np.repeat(v, n)
    th[:, 3] = np.tile(v, n)
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    E = b.n_events
    theta = tin(np.tile(th, (E, 1)))
    toff = tin(np.arange(E + 1, dtype=np.int64) * len(th))
    hits = (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))
    ms = {}
    for name, want in (("R", retina.WANT_R), ("RGH", retina.WANT_R | retina.WANT_GRAD | retina.WANT_HESS)):
        f = lambda: ctx.retina_response(2, b.plane_z, *hits, theta, toff, sigma=cfg["params"]["sigma_final"], want=want)
        f()
        torch.cuda.synchronize()
        ctx.retina_set_profiling(True)
        ctx.retina_profile_reset()
        for _ in range(5):
            f()
        torch.cuda.synchronize()
        pr = ctx.retina_get_profile()
        ctx.retina_set_profiling(False)
        ms[name] = pr["ms_hot"] / max(pr["calls"], 1)
    C = ms["RGH"] / ms["R"]
    print("C = %.3f (R %.3f ms, R + grad + Hess %.3f ms)" % (C, ms["R"], ms["RGH"]), flush=True)
    assert 1.0 < C < 3.0
