"""Pins of the grid-search Artificial Retina oracle (Section 2: the response at
every cell of a parameter grid, groups of high-response cells, one estimate
per group), through what the geometry fixes: symmetric neighbourhoods, exact
ties, the value of the grid against the independently pinned response
function, and the continuous maxima the multi-start procedure converges to."""
import numpy as np
import pytest

import oracle
from oracle.evaluate import _dist, match_tracks
from paper_1709_08610_amd import events

ZS = (20.0 + 730.0 * np.arange(26) / 25).astype(np.float32)


def _event3d(tracks, extra=None):
    """Noise-free hits exactly on the given (x0, y0, tx, ty) lines, one per plane,
    plus optional extra (x, y, plane) hits."""
    xs, ys, pls = [], [], []
    for x0, y0, tx, ty in tracks:
        xs.append(x0 + tx * ZS.astype(np.float64))
        ys.append(y0 + ty * ZS.astype(np.float64))
        pls.append(np.arange(ZS.size))
    if extra is not None:
        xs.append(extra[0])
        ys.append(extra[1])
        pls.append(extra[2])
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    return (cat(xs).astype(np.float32), cat(ys).astype(np.float32), cat(pls).astype(np.int32))


def _grid(n, lo, hi, sigma, R0):
    return dict(n=[n, n], lo=[lo, lo], hi=[hi, hi], sigma=sigma, R0=R0)


def _centres(g, axis):
    n, lo, hi = g["n"][axis], g["lo"][axis], g["hi"][axis]
    return (lo + (np.arange(n) + 0.5) * (hi - lo) / n).astype(np.float32).astype(np.float64)


def test_grid_values_are_the_response_at_cell_centres():
    """Step 2: each grid value is Eq. (1) at the cell centre (the lattice the seeds
    use), computed by the separately pinned response routine."""
    rng = np.random.default_rng(1)
    x, y, pl = _event3d([(0.01, -0.02, 0.0104, -0.0071), (0.0, 0.03, -0.0123, 0.0042)],
                        (rng.uniform(-5, 5, 40), rng.uniform(-5, 5, 40), rng.integers(0, 26, 40)))
    g = _grid(24, -0.024, 0.024, 0.4, 8.0)
    res = oracle.grid_search(2, ZS, x, y, pl, g)
    th = oracle.lattice(2, dict(sigma=[1.0], sigma_final=1.0, n_final_steps=0, n_polish=0, ls_trials=1,
                                armijo_c1=0.1, step_cap_sigmas=1.0, small_step_sigmas=0.0, conv_tol=1.0,
                                R0=1.0, d_merge=1.0, lattice_n=g["n"], lattice_lo=g["lo"], lattice_hi=g["hi"]))
    R, _, _ = oracle.response(2, ZS, x, y, pl, th, 0.4, want_derivs=False)
    np.testing.assert_allclose(res["R_grid"].ravel(), R, rtol=1e-13, atol=1e-300)


def test_track_at_a_cell_centre_one_peak_symmetric_estimate():
    """A noise-free track through the origin whose slopes are a cell centre: one
    peak, at that cell, with R = number of hits (every residual is rounding only);
    the neighbourhood is mirror-symmetric about the track, so the weighted
    estimate is the cell centre."""
    g = _grid(21, -0.021, 0.021, 0.375, 8.0)
    cx, cy = _centres(g, 0), _centres(g, 1)
    tx, ty = cx[13], cy[6]
    x, y, pl = _event3d([(0.0, 0.0, tx, ty)])
    res = oracle.grid_search(2, ZS, x, y, pl, g)
    assert list(res["cell"]) == [13 * 21 + 6]
    assert res["R"][0] == pytest.approx(26.0, abs=1e-6)
    np.testing.assert_allclose(res["theta"][0], [0.0, 0.0, tx, ty], atol=1e-9)
    assert res["members"][0] >= 1


def test_track_off_centre_estimate_moves_toward_truth():
    """The maximum is the nearest cell; the weighted mean of its neighbourhood lies
    between that cell's centre and the track, closer to the track."""
    g = _grid(21, -0.021, 0.021, 0.375, 8.0)
    cx, cy = _centres(g, 0), _centres(g, 1)
    step = 0.042 / 21
    tx, ty = cx[9] + 0.3 * step, cy[12] - 0.2 * step
    x, y, pl = _event3d([(0.0, 0.0, tx, ty)])
    res = oracle.grid_search(2, ZS, x, y, pl, g)
    assert list(res["cell"]) == [9 * 21 + 12]
    ex, ey = res["theta"][0, 2], res["theta"][0, 3]
    assert cx[9] < ex < tx and ty < ey < cy[12]
    assert abs(ex - tx) < 0.3 * step and abs(ey - ty) < 0.2 * step


def test_equal_neighbours_are_not_a_maximum():
    """The strict rule, on the 2D toy (Fig. 1 geometry) with planes symmetric about
    z = 0, where slope and offset decouple: a flat track exactly halfway between
    two slope cells gives those cells bit-identical responses (residuals +-z/64,
    dyadic values), so neither is a peak.  Moved slightly off the midpoint, the
    track has one peak; its estimate (x0, tx) = (beta, alpha) keeps the offset
    (mirror-symmetric offset neighbours) and pulls the slope toward the track."""
    zs = (np.arange(8) - 3.5).astype(np.float32)
    pl = np.arange(8, dtype=np.int32)
    # alpha centres (2i - 31)/64, beta centres (j - 16)/32: beta = 0.125 is cell 20
    g = dict(n=[32, 32], lo=[-0.5, -33 / 64], hi=[0.5, 31 / 64], sigma=0.3, R0=2.0)
    x = np.full(8, 0.125, np.float32)
    res = oracle.grid_search(1, zs, x, None, pl, g)
    G = res["R_grid"]
    assert G[15, 20] == G[16, 20] and G[15, 20] > 7.5
    assert len(res["cell"]) == 0
    x = (0.125 + 0.01 * zs.astype(np.float64)).astype(np.float32)
    res = oracle.grid_search(1, zs, x, None, pl, g)
    assert list(res["cell"]) == [16 * 32 + 20]
    assert res["theta"][0, 0] == pytest.approx(0.125, abs=1e-8)   # hits rounded to FP32
    assert 0.01 < res["theta"][0, 1] < 1 / 64


def test_threshold_empty_event_and_two_tracks_in_cell_order():
    g = _grid(40, -0.02, 0.02, 0.375, 8.0)
    x, y, pl = _event3d([])
    res = oracle.grid_search(2, ZS, x, y, pl, g)
    assert len(res["cell"]) == 0 and np.all(res["R_grid"] == 0)
    cx = _centres(g, 0)
    x, y, pl = _event3d([(0.0, 0.0, cx[30], cx[5]), (0.0, 0.0, cx[4], cx[33])])
    res = oracle.grid_search(2, ZS, x, y, pl, g)
    assert list(res["cell"]) == [4 * 40 + 33, 30 * 40 + 5]   # cell order, not response order
    g2 = dict(g, R0=26.5)                                     # above the 26 hits of a track
    assert len(oracle.grid_search(2, ZS, x, y, pl, g2)["cell"]) == 0


@pytest.mark.slow
def test_grid_peaks_lie_under_the_continuous_maxima_c1():
    """c1: every multi-start track (a continuous maximum of R, pinned elsewhere) with
    R clearly above R0 has a grid peak within a few cells (slope and offset are
    strongly correlated for planes at z = 1..8, so the discrete peak slides along the
    ridge by up to ~2 offset cells) whose response does not exceed the maximum's (a
    grid value in the basin of a maximum is at most its value), and the closest
    such peak is within 3% of it (the peak is narrower than two slope cells)."""
    cfg = events.load_config("c1")
    P = cfg["params"]
    for idx in range(2):
        b = events.make_batch(cfg, 1, start=idx)
        ev = b.event(0)
        res = oracle.find_tracks(b, P)
        g = dict(n=[960, 560], lo=[-1.2, -0.7], hi=[1.2, 0.7], sigma=P["sigma_final"], R0=P["R0"])
        gs = oracle.grid_search(1, b.plane_z, ev.x, None, ev.plane, g)
        step = np.array([1.4 / 560, 2.4 / 960])         # (x0, tx) cell sizes
        strong = res["R"] >= P["R0"] + 1.0
        for th, R in zip(res["theta"][strong], res["R"][strong]):
            cheb = (np.abs(gs["theta"] - th) / step).max(axis=1)
            near = cheb <= 3.0
            assert near.any(), "no grid peak next to a continuous maximum"
            assert gs["R"][near].max() <= R * (1 + 1e-9)
            assert gs["R"][np.argmin(cheb)] >= 0.97 * R
