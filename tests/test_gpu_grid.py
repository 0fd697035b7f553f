"""GPU parity of the grid-search Artificial Retina (retina_grid_search) against
the FP64 oracle (oracle.grid_search), through the C-ABI.

  * grid values: R within 1e-5 relative, widened by the FP32 forward error
    bound of the response (the rule of the response parity tests);
  * peaks: the same cells, except where the oracle's own decision is within
    that tolerance of flipping (a neighbour or R0 within the FP32 error of the
    cell's R); peak R within 1e-5 relative;
  * estimates: within 2e-5 of a cell (the weights carry FP32 relative errors
    of ~1e-6); n_members equal unless a neighbourhood value sits at R0."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events, retina

from gpu_util import assert_response_bounded, fp32_error_model

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


def _tol(R):
    return 3e-5 * np.abs(R) + 1e-6


def _cell_thetas(D, grid, cells):
    n0, n1 = grid["n"]
    i0, i1 = np.asarray(cells) // n1, np.asarray(cells) % n1
    c = lambda lo, hi, n, i: (lo + (i + 0.5) * (hi - lo) / n).astype(np.float32).astype(np.float64)
    v0 = c(grid["lo"][0], grid["hi"][0], n0, i0)
    v1 = c(grid["lo"][1], grid["hi"][1], n1, i1)
    z = np.zeros_like(v0)
    return np.stack([z, z, v0, v1], 1) if D == 2 else np.stack([v1, v0], 1)


def _margins(G, R0):
    """Per cell: R - max(in-grid neighbours) and R - R0 (oracle values)."""
    n0, n1 = G.shape
    P = np.full((n0 + 2, n1 + 2), -np.inf)
    P[1:-1, 1:-1] = G
    nb = np.full_like(G, -np.inf)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            if a or b:
                nb = np.maximum(nb, P[1 + a:1 + a + n0, 1 + b:1 + b + n1])
    return G - nb, G - R0


def _compare_event(D, zp, ev, grid, gpu_tracks, gpu_grid, ref, sample=None, seed=0):
    """One event: GPU grid, peaks and estimates against the oracle's."""
    n0, n1 = grid["n"]
    Gref = ref["R_grid"]
    Ggpu = gpu_grid.reshape(n0, n1).astype(np.float64)
    cells = np.arange(n0 * n1)
    if sample is not None and sample < cells.size:
        cells = np.random.default_rng(seed).choice(cells, sample, replace=False)
    th = _cell_thetas(D, grid, cells)
    model = fp32_error_model(D, zp, ev.x, ev.y, ev.plane, th, grid["sigma"])
    assert_response_bounded(Ggpu.ravel()[cells], Gref.ravel()[cells], None, None, None, None, model,
                            ev.n_hits, grid["sigma"], float(np.max(np.abs(zp))))
    # peak decisions
    mn, m0 = _margins(Gref, grid["R0"])
    tol = _tol(Gref)
    g_cells = np.asarray(gpu_tracks["seed_index"], np.int64)
    r_cells = ref["cell"]
    assert np.all(np.diff(g_cells) > 0), "GPU peaks not in cell order"
    diff = np.setxor1d(g_cells, r_cells)
    marginal = (np.abs(mn.ravel()[diff]) <= tol.ravel()[diff]) | (np.abs(m0.ravel()[diff]) <= tol.ravel()[diff])
    assert marginal.all(), "peak decisions differ at cells %s (oracle margins %s)" % (
        diff[~marginal][:5], mn.ravel()[diff[~marginal]][:5])
    common, gi, ri = np.intersect1d(g_cells, r_cells, return_indices=True)
    np.testing.assert_allclose(gpu_tracks["R"][gi], ref["R"][ri], rtol=1e-5, atol=1e-6)
    step = np.array([(grid["hi"][k] - grid["lo"][k]) / grid["n"][k] for k in (0, 1)])
    span = np.array([0, 0, step[0], step[1]]) if D == 2 else np.array([step[1], step[0]])
    dth = np.abs(gpu_tracks["theta"][gi, :2 * D] - ref["theta"][ri])
    assert np.all(dth <= 2e-5 * span + 1e-12), "estimate error %s cells" % (dth / np.maximum(span, 1e-30)).max()
    near_R0 = np.zeros(len(common), bool)
    for k, c in enumerate(common):
        i0, i1 = divmod(int(c), n1)
        win = Gref[max(i0 - 1, 0):i0 + 2, max(i1 - 1, 0):i1 + 2]
        near_R0[k] = np.any(np.abs(win - grid["R0"]) <= _tol(win))
    same = gpu_tracks["n_members"][gi] == ref["members"][ri]
    assert np.all(same | near_R0)
    return len(common), len(diff)


def _run(ctx, b, grid, mem="host"):
    if mem == "host":
        return ctx.retina_grid_search(b.meas_dim, b.plane_z, b.event_offsets, b.x, b.y, b.plane, grid,
                                      want_grid=True)
    import torch
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    res = ctx.retina_grid_search(b.meas_dim, b.plane_z, t(b.event_offsets), t(b.x), t(b.y), t(b.plane), grid,
                                 want_grid=True)
    torch.cuda.synchronize()
    toff = res["track_offsets"].cpu().numpy()
    tr = res["tracks_bytes"].cpu().numpy()[: int(toff[-1]) * 48].view(retina.TRACK_DTYPE)
    return dict(tracks=tr, track_offsets=toff, R_grid=res["R_grid"].cpu().numpy())


def _check_batch(ctx, b, grid, mem="host", sample=3000):
    res = _run(ctx, b, grid, mem)
    toff = res["track_offsets"]
    n_pk = 0
    for e in range(b.n_events):
        ev = b.event(e)
        ref = oracle.grid_search(b.meas_dim, b.plane_z, ev.x, ev.y, ev.plane, grid)
        tr = res["tracks"][toff[e]:toff[e + 1]]
        nc, nd = _compare_event(b.meas_dim, b.plane_z, ev, grid, tr, res["R_grid"][e], ref, sample=sample, seed=e)
        n_pk += nc
        _say("  event %d: %d hits, %d peaks agree, %d marginal decisions" % (e, ev.n_hits, nc, nd))
    return res, n_pk


def c2_grid(n=120, sigma=None, R0=8.0):
    """A grid over the c2/c3 slope box; default sigma = half a cell at the last plane."""
    step = 0.6 / n
    return dict(n=[n, n], lo=[-0.3, -0.3], hi=[0.3, 0.3], sigma=sigma or 0.5 * step * 750.0, R0=R0)


def test_grid_c2_event_coarse(ctx):
    _say("grid search: c2 event, 120 x 120 cells")
    b = events.make_batch(events.load_config("c2"))
    _, n = _check_batch(ctx, b, c2_grid(120))
    assert n > 100


def test_grid_c3_uneven_batch_device_memory(ctx):
    _say("grid search: c3 events 0..5 (uneven), 64 x 64 cells, device memory")
    b = events.make_batch(events.load_config("c3"), 6)
    _check_batch(ctx, b, c2_grid(64), mem="device")


def test_grid_c1_two_dimensional_toy(ctx):
    _say("grid search: c1 (meas_dim 1), 400 x 400 cells at sigma_final")
    cfg = events.load_config("c1")
    P = cfg["params"]
    b = events.make_batch(cfg)
    grid = dict(n=[400, 400], lo=list(P["lattice_lo"]), hi=list(P["lattice_hi"]), sigma=P["sigma_final"],
                R0=P["R0"])
    _, n = _check_batch(ctx, b, grid)
    assert n >= 5


def test_grid_c2_event_full_resolution(ctx):
    """The workload of the grid-vs-multi-start comparison: a c2 event on the
    600 x 600 grid of 1e-3 slope resolution; the oracle evaluates every cell
    (peak decisions and estimates), the error-bounded R check samples 4000."""
    _say("grid search: c2 event, 600 x 600 cells (1e-3 resolution)")
    b = events.make_batch(events.load_config("c2"))
    _, n = _check_batch(ctx, b, c2_grid(600), sample=4000)
    assert n > 150


def test_grid_edges(ctx):
    """Ragged grids (a partial last chunk and round), a 1 x 1 grid (no
    neighbours), events without hits inside a batch, host and device memory
    agreeing bit for bit, the capacity error and rejected arguments."""
    _say("grid search: edge cases")
    cfg = events.load_config("c3")
    evs = [events.make_event(cfg, 0, events.plane_z(cfg))]
    empty = events.Event(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32),
                         np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros(0, np.int32))
    b = events.batch_from_events(2, events.plane_z(cfg), [empty, evs[0], empty])
    grid = dict(n=[97, 101], lo=[-0.3, -0.3], hi=[0.3, 0.3], sigma=2.5, R0=8.0)
    res, _ = _check_batch(ctx, b, grid)
    toff = res["track_offsets"]
    assert toff[1] == 0 and toff[3] == toff[2] and toff[2] > 0
    assert np.all(res["R_grid"][0] == 0) and np.all(res["R_grid"][2] == 0)
    dres = _run(ctx, b, grid, mem="device")
    assert np.array_equal(dres["R_grid"], res["R_grid"])
    assert np.array_equal(dres["track_offsets"], toff)
    assert dres["tracks"].tobytes() == res["tracks"].tobytes()
    # 1 x 1: the only cell is a peak iff it reaches R0
    one = dict(n=[1, 1], lo=[-0.3, -0.3], hi=[0.3, 0.3], sigma=400.0, R0=1.0)
    r1 = _run(ctx, b, one)
    assert list(np.diff(r1["track_offsets"])) == [0, 1, 0]
    assert r1["tracks"][0]["theta"][2] == pytest.approx(0.0, abs=1e-7)
    # capacity
    with pytest.raises(retina.RetinaError) as ei:
        ctx.retina_grid_search(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, grid, capacity=1)
    assert ei.value.code == retina.ERR_CAPACITY and ei.value.required == int(toff[-1])
    for bad in (dict(grid, R0=0.0), dict(grid, sigma=-1.0), dict(grid, n=[0, 5]), dict(grid, lo=[0.3, -0.3]),
                dict(grid, hi=[0.3, float("nan")])):
        with pytest.raises(retina.RetinaError) as ei:
            ctx.retina_grid_search(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, bad)
        assert ei.value.code == retina.ERR_INVALID_ARG
