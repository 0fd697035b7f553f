"""Pins of the oracle's multi-start procedure (Algorithm 1, Section 3).

The procedure is a heuristic, so it is pinned through what the mathematics
fixes: the Newton direction of a positive-definite model is the linear-solve
solution, a converged maximum is a weighted least-squares fixed point, a huge
bandwidth turns the maximum into the ordinary least-squares line, the
maxima found from seeds are maxima of a dense brute-force grid, and the
cluster step follows hand-worked examples."""
import numpy as np
import pytest

import oracle
from oracle.evaluate import _dist, match_tracks
from paper_1709_08610_amd import events


# ----------------------------------------------------------------- Newton-CG
def _spd(rng, n):
    a = rng.normal(size=(n, n))
    return a @ a.T + n * np.eye(n)


@pytest.mark.parametrize("n", [2, 4])
def test_newton_cg_solves_pd_system(n):
    """With -H positive definite and a tiny gradient, CG runs to convergence and the
    direction is the Newton step (-H)^-1 g, whatever the scaling."""
    rng = np.random.default_rng(n)
    for _ in range(10):
        A = _spd(rng, n)
        H = -A
        g = rng.normal(size=n) * 1e-12
        ds = rng.uniform(0.5, 400.0, n)
        p, pn, neg = oracle.newton_cg(g, H, ds, sigma=1.0, cap=2.0)
        assert not neg
        np.testing.assert_allclose(p, np.linalg.solve(A, g), rtol=1e-5)
        assert pn == pytest.approx(np.linalg.norm(ds * p), rel=1e-12)


def test_newton_cg_negative_curvature_first_direction():
    """H positive definite (R convex there): the step is steepest ascent in scaled
    coordinates with length one bandwidth."""
    rng = np.random.default_rng(3)
    A = _spd(rng, 4)
    g = rng.normal(size=4)
    ds = np.array([1.0, 1.0, 400.0, 400.0])
    sigma = 0.7
    p, pn, neg = oracle.newton_cg(g, A, ds, sigma=sigma, cap=2.0)
    assert neg
    b = g / ds
    np.testing.assert_allclose(ds * p, sigma * b / np.linalg.norm(b), rtol=1e-14)
    assert pn == pytest.approx(sigma, rel=1e-14)


def test_newton_cg_cap():
    rng = np.random.default_rng(4)
    A = _spd(rng, 4) * 1e-6  # very flat: Newton step huge
    g = rng.normal(size=4)
    ds = np.ones(4)
    p, pn, neg = oracle.newton_cg(g, -A, ds, sigma=0.5, cap=2.0)
    assert not neg
    assert pn == pytest.approx(1.0, rel=1e-12)
    assert np.linalg.norm(p) == pytest.approx(1.0, rel=1e-12)
    # same direction as the (truncated) CG iterate: ascent direction
    assert g @ p > 0


def test_newton_cg_zero_gradient():
    p, pn, neg = oracle.newton_cg(np.zeros(4), -np.eye(4), np.ones(4), 1.0, 2.0)
    assert np.all(p == 0) and pn == 0 and not neg


# ------------------------------------------------------------------- lattice
def test_lattice_cell_centred_row_major():
    P = events.load_config("c2")["params"]
    L = oracle.lattice(2, P)
    n = P["lattice_n"][0]
    assert L.shape == (n * n, 4)
    assert np.all(L[:, :2] == 0)
    step = 0.6 / n
    # index 1 moves the fast dimension (ty); index n moves tx
    assert L[1, 3] - L[0, 3] == pytest.approx(step, rel=1e-6)
    assert L[n, 2] - L[0, 2] == pytest.approx(step, rel=1e-6)
    lo, hi = float(np.float32(-0.3)), float(np.float32(0.3))  # the box edges are FP32 inputs
    assert L[0, 2] == np.float32(lo + 0.5 * (hi - lo) / n)
    assert np.all(L == L.astype(np.float32))  # FP32 values
    # symmetric cell centres
    np.testing.assert_allclose(np.sort(np.unique(L[:, 2])), -np.sort(np.unique(L[:, 2]))[::-1], atol=1e-7)


def test_lattice_meas_dim_one_order():
    P = events.load_config("c1")["params"]
    L = oracle.lattice(1, P)
    # dims (tx, x0): theta = (x0, tx); x0 is the fast index
    assert L[1, 0] > L[0, 0] and L[1, 1] == L[0, 1]
    assert L[30, 1] > L[0, 1]


# -------------------------------------------------------------------- merge
def test_merge_hand_example():
    """Leaders in decreasing R, ties to the lower seed index, each candidate joins the
    FIRST leader within d_merge; unconverged and below-threshold seeds are dropped."""
    th = np.zeros((7, 4))
    th[:, 0] = [0.0, 0.001, 0.0, 1.0, 0.02, 5.0, 0.0]  # x0 offsets (mm)
    R = np.array([10.0, 12.0, 12.0, 9.0, 11.0, 20.0, 30.0])
    fl = np.array([1, 1, 1, 1, 1, 1, 0], np.int32)  # seed 6 not converged
    R0 = 9.5  # drops seed 3
    leaders, members = oracle.merge(2, th, R, fl, R0, 0.03, 20.0, 750.0)
    # order: 5 (R 20), then 1 and 2 (R 12, tie -> 1 first), 4 (11), 0 (10)
    # 5 founds; 1 founds (x0 0.001 far from 5.0); 2 joins 1; 4: |0.02-0.001| <= 0.03 joins 1; 0 joins 1
    assert list(leaders) == [5, 1]
    assert list(members) == [1, 4]


def test_merge_joins_first_leader_not_nearest():
    th = np.zeros((3, 2))
    th[:, 0] = [0.0, 0.05, 0.03]  # D=1: (x0, tx)
    R = np.array([10.0, 9.0, 8.0])
    fl = np.ones(3, np.int32)
    leaders, members = oracle.merge(1, th, R, fl, 1.0, 0.035, 1.0, 8.0)
    # seed 2 is 0.03 from leader 0 and 0.02 from leader 1: it joins leader 0 (created first)
    assert list(leaders) == [0, 1]
    assert list(members) == [2, 1]


def test_merge_distance_uses_end_planes():
    # two lines that coincide at z = 20 but separate by 0.04 at z = 750
    th = np.array([[0.0, 0.0, 0.0, 0.0], [-0.04 / 730 * 20, 0.0, 0.04 / 730, 0.0]])
    R = np.array([10.0, 9.0])
    fl = np.ones(2, np.int32)
    leaders, _ = oracle.merge(2, th, R, fl, 1.0, 0.03, 20.0, 750.0)
    assert len(leaders) == 2
    leaders, _ = oracle.merge(2, th, R, fl, 1.0, 0.05, 20.0, 750.0)
    assert len(leaders) == 1


def test_merge_empty():
    leaders, members = oracle.merge(2, np.zeros((0, 4)), np.zeros(0), np.zeros(0, np.int32), 1.0, 0.03, 20, 750)
    assert len(leaders) == 0


# ----------------------------------------------------------- ascent results
def _single_track_batch(theta, zp, sd=0.0, seed=0, noise=0):
    rng = np.random.default_rng(seed)
    z = zp.astype(np.float64)
    x = (theta[0] + theta[2] * z + rng.normal(0, sd, z.size)).astype(np.float32) if sd else \
        (theta[0] + theta[2] * z).astype(np.float32)
    y = (theta[1] + theta[3] * z + rng.normal(0, sd, z.size)).astype(np.float32) if sd else \
        (theta[1] + theta[3] * z).astype(np.float32)
    pl = np.arange(z.size, dtype=np.int32)
    if noise:
        x = np.r_[x, rng.uniform(-40, 40, noise).astype(np.float32)]
        y = np.r_[y, rng.uniform(-40, 40, noise).astype(np.float32)]
        pl = np.r_[pl, rng.integers(0, z.size, noise).astype(np.int32)]
    ev = events.Event(x, y, pl, np.zeros(x.size, np.int32), theta[None, :], np.array([z.size], np.int32))
    return events.batch_from_events(2, zp, [ev])


def test_ascent_recovers_noise_free_track():
    """Seeds inside the basin of an isolated noise-free track end exactly on it."""
    cfg = events.load_config("c2")
    zp = events.plane_z(cfg)
    th = np.array([0.03125, -0.015625, 0.1, -0.2])
    b = _single_track_batch(th, zp)
    # the hits are FP32: the exact maximum is the FP64 least-squares line through them
    z = zp.astype(np.float64)
    A = np.c_[np.ones_like(z), z]
    sx = np.linalg.lstsq(A, b.x.astype(np.float64), rcond=None)[0]
    sy = np.linalg.lstsq(A, b.y.astype(np.float64), rcond=None)[0]
    star = np.array([sx[0], sy[0], sx[1], sy[1]])
    rng = np.random.default_rng(2)
    seeds = np.zeros((16, 4))
    seeds[:, 2] = th[2] + rng.uniform(-0.004, 0.004, 16)
    seeds[:, 3] = th[3] + rng.uniform(-0.004, 0.004, 16)
    res = oracle.find_tracks(b, cfg["params"], seeds=seeds, seed_offsets=np.array([0, 16]))
    assert np.all(res["seed_flags"] & oracle.CONVERGED)
    np.testing.assert_allclose(res["seed_theta"], np.broadcast_to(star, (16, 4)), rtol=1e-9, atol=1e-12)
    assert len(res["R"]) == 1 and res["members"][0] == 16
    # FP32 rounding leaves residuals ~1e-5 mm: R = 26 - O(r^2/sigma^2)
    assert res["R"][0] == pytest.approx(26.0, rel=1e-7)


def test_converged_maximum_is_weighted_least_squares_fixed_point():
    """At a stationary point, theta* is the weighted least-squares line with weights
    e_k(theta*) (the Welsch M-estimator / IRLS fixed point), solved with lstsq."""
    cfg = events.load_config("c2")
    b = events.make_batch(cfg, 1)
    ev = b.event(0)
    # seeds next to a handful of true tracks, to keep the test fast
    seeds = np.zeros((12, 4))
    seeds[:, 2:] = ev.truth[:12, 2:] + 0.001
    res = oracle.find_tracks(b, cfg["params"], seeds=seeds, seed_offsets=np.array([0, 12]))
    z = b.plane_z.astype(np.float64)[ev.plane]
    sig = cfg["params"]["sigma_final"]
    checked = 0
    for i in range(12):
        if not res["seed_flags"][i] & oracle.CONVERGED:
            continue
        t = res["seed_theta"][i]
        rx = ev.x - t[0] - t[2] * z
        ry = ev.y - t[1] - t[3] * z
        w = np.sqrt(np.exp(-(rx ** 2 + ry ** 2) / np.float32(sig) ** 2))
        A = np.c_[np.ones_like(z), z] * w[:, None]
        sx = np.linalg.lstsq(A, ev.x * w, rcond=None)[0]
        sy = np.linalg.lstsq(A, ev.y * w, rcond=None)[0]
        np.testing.assert_allclose([sx[0], sy[0]], t[:2], atol=1e-9)
        np.testing.assert_allclose([sx[1], sy[1]], t[2:], atol=1e-11)
        checked += 1
    assert checked >= 10


def test_huge_bandwidth_gives_ordinary_least_squares():
    """sigma >> residuals: argmax R -> the OLS line (error O(r^2/sigma^2))."""
    zp = events.plane_z(events.load_config("c2"))
    th = np.array([0.05, -0.02, 0.12, 0.07])
    b = _single_track_batch(th, zp, sd=0.012, seed=3)
    z = zp.astype(np.float64)
    A = np.c_[np.ones_like(z), z]
    sx = np.linalg.lstsq(A, b.x.astype(np.float64), rcond=None)[0]
    sy = np.linalg.lstsq(A, b.y.astype(np.float64), rcond=None)[0]
    ols = np.array([sx[0], sy[0], sx[1], sy[1]])
    ev = b.event(0)
    for sigma, tol in [(100.0, 1e-7), (1000.0, 1e-9)]:
        out, R, step, pd = oracle.polish(2, zp, ev.x, ev.y, ev.plane, th, sigma, 6)
        assert pd[0]
        np.testing.assert_allclose(out[0], ols, rtol=0, atol=tol * np.abs(ols).max() * 10)


# ---------------------------------------------------- brute-force grid (c1)
def _grid_maxima(b, sigma, R0, d_merge, n_grid, lo, hi):
    """Strict 8-neighbour maxima of R on a dense (tx, x0) grid, each Newton-polished
    in FP64; converged maxima with R >= R0, deduplicated within d_merge."""
    ev = b.event(0)
    ta = np.linspace(lo[0], hi[0], n_grid[0])
    xb = np.linspace(lo[1], hi[1], n_grid[1])
    TT, XX = np.meshgrid(ta, xb, indexing="ij")
    th = np.stack([XX.ravel(), TT.ravel()], axis=1)
    R, _, _ = oracle.response(1, b.plane_z, ev.x, None, ev.plane, th, sigma, want_derivs=False)
    G = R.reshape(n_grid)
    core = G[1:-1, 1:-1]
    is_max = np.ones_like(core, bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di or dj:
                is_max &= core > G[1 + di:G.shape[0] - 1 + di, 1 + dj:G.shape[1] - 1 + dj]
    is_max &= core >= 0.25 * R0
    ii, jj = np.nonzero(is_max)
    pts = np.stack([XX[ii + 1, jj + 1], TT[ii + 1, jj + 1]], axis=1)
    out, Rp, step, pd = oracle.polish(1, b.plane_z, ev.x, None, ev.plane, pts, sigma, 30)
    ok = pd & (step <= 1e-9) & (Rp >= R0)
    out, Rp = out[ok], Rp[ok]
    order = np.argsort(-Rp, kind="stable")
    keep = []
    for k in order:
        if all(_dist(1, out[k], out[j], b.plane_z.min(), b.plane_z.max())[0, 0] > d_merge for j in keep):
            keep.append(k)
    return out[keep], Rp[keep]


@pytest.mark.slow
def test_multistart_maxima_are_brute_force_maxima_c1():
    """c1: every track the multi-start procedure returns is a maximum of R found by a
    dense brute-force grid (800 x 800, twice the nominal 400 x 400 since the peak width
    along the slope, 0.0031, is below the nominal grid step), with the same R; and every
    grid maximum that lies near a true track is found."""
    cfg = events.load_config("c1")
    P = cfg["params"]
    for idx in range(3):
        b = events.make_batch(cfg, 1, start=idx)
        res = oracle.find_tracks(b, P)
        bf, Rbf = _grid_maxima(b, P["sigma_final"], P["R0"], P["d_merge"], (800, 800),
                               (-1.2, -0.7), (1.2, 0.7))
        f2b, b2f, d = match_tracks(1, res["theta"], bf, 1e-6, 1.0, 8.0)
        assert np.all(f2b >= 0), "a multi-start track is not a grid maximum"
        # the multi-start stops at a last step <= 1e-3 sigma (quadratic convergence leaves
        # ~1e-6 sigma), the grid polish runs to 1e-9: R agrees to second order in that gap
        np.testing.assert_allclose(res["R"], Rbf[f2b], rtol=1e-7)
        ev = b.event(0)
        near_true = _dist(1, bf, ev.truth, 1.0, 8.0).min(axis=1) <= cfg["match_tol"]
        # the converse is the method's efficiency, not an identity: multi-start may miss a
        # maximum no seed flows to (crossing lines in c1); most must be found
        assert np.mean(b2f[near_true] >= 0) >= 0.8, "too many grid maxima on true tracks missed"


def _toy2d_event(tracks, zs, sd, n_noise, seed, noise_lo=-2.0, noise_hi=2.0):
    rng = np.random.default_rng(seed)
    xs, pls = [], []
    for x0, tx in tracks:
        xs.append(x0 + tx * zs + rng.normal(0, sd, zs.size))
        pls.append(np.arange(zs.size))
    xs.append(rng.uniform(noise_lo, noise_hi, n_noise))
    pls.append(rng.integers(0, zs.size, n_noise))
    x = np.concatenate(xs).astype(np.float32)
    pl = np.concatenate(pls).astype(np.int32)
    ev = events.Event(x, None, pl, np.zeros(x.size, np.int32), np.array(tracks), np.full(len(tracks), zs.size))
    return events.batch_from_events(1, zs.astype(np.float32), [ev])


def test_fig1_two_tracks_two_maxima():
    """Fig. 1: two 10-hit tracks plus 20 uniform noise hits at sigma = 0.02 give exactly
    two response maxima well above the noise, each next to a true track."""
    zs = np.arange(1, 11, dtype=np.float64)
    tracks = [(0.1, 0.3), (0.4, -0.2)]
    b = _toy2d_event(tracks, zs, 0.005, 20, seed=5)
    bf, Rbf = _grid_maxima(b, 0.02, 5.0, 0.02, (600, 600), (-1.0, -1.0), (1.0, 1.0))
    assert len(bf) == 2
    d = _dist(1, bf, np.array(tracks), 1.0, 10.0)
    assert np.all(d.min(axis=1) < 0.03)


@pytest.mark.parametrize("sigma,expect", [(0.1, 1), (0.03, 2)])
def test_fig2_bandwidth_merges_or_resolves_close_tracks(sigma, expect):
    """Fig. 2: two parallel 20-hit tracks 0.08 apart with N(0, 0.01) hit noise: a large
    bandwidth (0.1) merges them into one maximum, a bandwidth near the hit noise (0.03)
    resolves two."""
    zs = np.arange(1, 21, dtype=np.float64) * 0.05
    tracks = [(0.0, 0.5), (0.08, 0.5)]
    b = _toy2d_event(tracks, zs, 0.01, 0, seed=7)
    # R0 = 17 of 20 hits: above the diagonal maxima that cross from one track to the other
    bf, Rbf = _grid_maxima(b, sigma, 17.0, 1e-3, (301, 301), (0.3, -0.2), (0.7, 0.3))
    assert len(bf) == expect


# ---------------------------------------------------------------- evaluation
def test_match_greedy_nearest_first():
    truth = np.array([[0.0, 0.0, 0.1, 0.1], [0.0, 0.0, -0.1, 0.0]])
    found = np.array([[0.01, 0.0, 0.1, 0.1], [0.001, 0.0, 0.1, 0.1], [5.0, 0, 0, 0]])
    f2t, t2f, d = match_tracks(2, found, truth, 0.06, 20.0, 750.0)
    assert list(t2f) == [1, -1]
    assert list(f2t) == [-1, 0, -1]
    st = oracle.efficiency(2, found, truth, np.array([5, 1]), 0.06, 20.0, 750.0)
    assert st["n_true_rec"] == 1 and st["n_matched"] == 1
    assert st["n_clone"] == 1 and st["n_fake"] == 1
