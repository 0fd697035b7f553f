"""Pins of the oracle's response, gradient and Hessian (Eq. (1), Section 3).

Each test checks the oracle against something other than its own formula:
hand-derived values, a closed-form maximum, finite differences and exact
invariances of the arithmetic."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
ZP = np.array([20.0, 100.0, 250.0, 400.0, 750.0], np.float32)


def _line_hits(theta, zs, dx, dy):
    x0, y0, tx, ty = theta
    x = np.array([x0 + tx * z + a for z, a in zip(zs, dx)], np.float32)
    y = np.array([y0 + ty * z + b for z, b in zip(zs, dy)], np.float32)
    return x, y


def test_golden_single_hit_values():
    """One hit at a known in-plane distance: R = exp(-d^2/sigma^2) (hand values)."""
    g = json.load(open(GOLD))
    sigma = 0.25  # power of two so that d = sigma*sqrt(c) stays exact in the ratio
    z = np.array([3.0], np.float32)
    for case in g["cases"]:
        d = sigma * np.sqrt(case["d_over_sigma_sq"])
        # the line x = 0 at the hit's plane; hit displaced by d along x (exactly representable
        # is not needed: compare against exp of the FP32 hit's own distance at 1e-7)
        x = np.array([d], np.float32)
        y = np.array([0.0], np.float32)
        R, gr, h = oracle.response(2, z, x, y, np.array([0], np.int32), [0, 0, 0, 0], sigma)
        assert R[0] == pytest.approx(case["R"], rel=2e-7, abs=1e-12)
    # gradient of the ln 2 case
    d = np.float32(sigma * np.sqrt(np.log(2.0)))
    R, gr, h = oracle.response(2, z, np.array([d]), np.array([0.0], np.float32), np.array([0], np.int32),
                               [0, 0, 0, 0], sigma)
    assert gr[0, 0] * sigma == pytest.approx(g["gradient_x0_times_sigma_for_d_sigma_sqrt_ln2"], rel=2e-7)
    assert gr[0, 1] == 0.0


def test_noise_free_track_closed_form():
    """Hits exactly on theta*: R = k, grad = 0, Hess = -(2/sigma^2) * [[k, sum z], [sum z, sum z^2]]
    in each coordinate block, zero across blocks (Eq. (1) maximum)."""
    zs = ZP.astype(np.float64)
    # choose a line whose hits are exact in FP32: dyadic parameters and integer z
    th = np.array([0.5, -0.25, 0.125, -0.0625])
    x, y = _line_hits(th, zs, np.zeros(5), np.zeros(5))
    assert np.all(x.astype(np.float64) == th[0] + th[2] * zs)
    sigma = 0.03
    R, g, h = oracle.response(2, ZP, x, y, np.arange(5, dtype=np.int32), th, sigma)
    H = oracle.unpack_hess(h, 4)[0]
    k, sz, szz = 5.0, zs.sum(), (zs ** 2).sum()
    c = -2.0 / sigma ** 2
    expect = c * np.array([[k, 0, sz, 0], [0, k, 0, sz], [sz, 0, szz, 0], [0, sz, 0, szz]])
    assert R[0] == k
    assert np.all(g == 0.0)
    np.testing.assert_allclose(H, expect, rtol=1e-14)


def test_max_at_noise_free_track_is_global():
    """Every term of Eq. (1) is <= 1, so R(theta*) = k is the global maximum and any
    other hits can only add to it: R(theta*) >= k."""
    rng = np.random.default_rng(1)
    zs = ZP.astype(np.float64)
    th = np.array([0.5, -0.25, 0.125, -0.0625])
    x, y = _line_hits(th, zs, np.zeros(5), np.zeros(5))
    nx = rng.uniform(-40, 40, 30).astype(np.float32)
    ny = rng.uniform(-40, 40, 30).astype(np.float32)
    npl = rng.integers(0, 5, 30).astype(np.int32)
    X = np.r_[x, nx]
    Y = np.r_[y, ny]
    PL = np.r_[np.arange(5, dtype=np.int32), npl]
    R_star, _, _ = oracle.response(2, ZP, X, Y, PL, th, 0.03, want_derivs=False)
    assert R_star[0] >= 5.0
    thetas = th + rng.normal(0, 1e-3, (200, 4)) * np.array([1, 1, 1e-2, 1e-2])
    R_pert, _, _ = oracle.response(2, ZP, x, y, np.arange(5, dtype=np.int32), thetas, 0.03, want_derivs=False)
    assert np.all(R_pert <= 5.0)


def _random_event(D, n=60, seed=3):
    rng = np.random.default_rng(seed)
    pl = rng.integers(0, 5, n).astype(np.int32)
    x = rng.normal(0, 0.5, n).astype(np.float32)
    y = rng.normal(0, 0.5, n).astype(np.float32) if D == 2 else None
    return x, y, pl


@pytest.mark.parametrize("D", [1, 2])
def test_finite_difference_gradient_and_hessian(D):
    """Central differences of R reproduce grad R; of grad R reproduce Hess R."""
    x, y, pl = _random_event(D)
    zp = np.array([0.5, 1.0, 1.5, 2.0, 2.5], np.float32)
    npar = 2 * D
    rng = np.random.default_rng(7)
    sigma = 0.4
    for _ in range(5):
        th = rng.normal(0, 0.3, npar)
        R, g, h = oracle.response(D, zp, x, y, pl, th, sigma)
        H = oracle.unpack_hess(h, npar)[0]
        eps = 1e-5
        for a in range(npar):
            tp = th.copy(); tp[a] += eps
            tm = th.copy(); tm[a] -= eps
            Rp, gp, _ = oracle.response(D, zp, x, y, pl, tp, sigma)
            Rm, gm, _ = oracle.response(D, zp, x, y, pl, tm, sigma)
            fd_g = (Rp[0] - Rm[0]) / (2 * eps)
            assert fd_g == pytest.approx(g[0, a], rel=1e-7, abs=1e-7 * np.abs(g).max())
            fd_h = (gp[0] - gm[0]) / (2 * eps)
            np.testing.assert_allclose(fd_h, H[a], rtol=1e-6, atol=1e-7 * np.abs(H).max())


def test_hessian_symmetric_and_packing():
    x, y, pl = _random_event(2)
    zp = np.array([0.5, 1.0, 1.5, 2.0, 2.5], np.float32)
    th = np.array([[0.1, -0.2, 0.05, 0.3], [0.0, 0.0, 0.0, 0.0]])
    R, g, h = oracle.response(2, zp, x, y, pl, th, 0.5)
    assert h.shape == (2, 10)
    H = oracle.unpack_hess(h, 4)
    np.testing.assert_array_equal(H, np.transpose(H, (0, 2, 1)))


def test_shear_invariance():
    """x -> x + a + b z together with (x0, tx) -> (x0 + a, tx + b) leaves R, g, H unchanged
    (the residuals are unchanged).  Dyadic a, b keep the shifted hits exact."""
    x, y, pl = _random_event(2, seed=11)
    x = (np.round(x * 1024) / 1024).astype(np.float32)  # coarse dyadic grid: the shift is exact
    zp = np.array([1.0, 2.0, 3.0, 4.0, 5.0], np.float32)
    a, b = 0.5, 0.25
    xs = (x.astype(np.float64) + a + b * zp[pl]).astype(np.float32)
    assert np.all(xs.astype(np.float64) == x.astype(np.float64) + a + b * zp[pl])
    th = np.array([0.1, -0.2, 0.05, 0.3])
    R1, g1, h1 = oracle.response(2, zp, x, y, pl, th, 0.5)
    R2, g2, h2 = oracle.response(2, zp, xs, y, pl, th + np.array([a, 0, b, 0]), 0.5)
    np.testing.assert_allclose(R2, R1, rtol=1e-13)
    np.testing.assert_allclose(g2, g1, rtol=1e-10, atol=1e-12 * np.abs(g1).max())
    np.testing.assert_allclose(h2, h1, rtol=1e-10, atol=1e-12 * np.abs(h1).max())


@pytest.mark.parametrize("m", [-3, 2, 5])
def test_power_of_two_scaling(m):
    """Scaling hit coordinates, offsets, slopes and sigma by 2^m leaves R bit-identical;
    g scales by 2^-m and H by 2^-2m (all exactly, since the scale is a power of two)."""
    x, y, pl = _random_event(2, seed=5)
    zp = np.array([0.5, 1.0, 1.5, 2.0, 2.5], np.float32)
    th = np.array([0.1, -0.2, 0.05, 0.3])
    s = 2.0 ** m
    R1, g1, h1 = oracle.response(2, zp, x, y, pl, th, 0.5)
    R2, g2, h2 = oracle.response(2, zp, (x * s).astype(np.float32), (y * s).astype(np.float32), pl,
                                 th * s, 0.5 * s)
    np.testing.assert_array_equal(R2, R1)
    np.testing.assert_array_equal(g2, g1 / s)
    np.testing.assert_array_equal(h2, h1 / s ** 2)


def test_hit_permutation_changes_only_rounding():
    b = events.make_batch(events.load_config("c2"), 1)
    ev = b.event(0)
    perm = np.random.default_rng(0).permutation(ev.n_hits)
    th = np.array([[0.0, 0.0, 0.1, -0.05], [0.01, 0.02, -0.2, 0.1]])
    R1, g1, h1 = oracle.response(2, b.plane_z, ev.x, ev.y, ev.plane, th, 1.0)
    R2, g2, h2 = oracle.response(2, b.plane_z, ev.x[perm], ev.y[perm], ev.plane[perm], th, 1.0)
    np.testing.assert_allclose(R2, R1, rtol=1e-12)


def test_meas_dim_one_matches_two_dim_with_far_y():
    """D = 1 is the x-block of D = 2: with every y residual zero, R and the x-block of
    g and H agree."""
    x, _, pl = _random_event(1, seed=9)
    zp = np.array([1.0, 2.0, 3.0, 4.0, 5.0], np.float32)
    th1 = np.array([0.1, 0.05])
    th2 = np.array([0.1, 0.0, 0.05, 0.0])
    R1, g1, h1 = oracle.response(1, zp, x, None, pl, th1, 0.5)
    R2, g2, h2 = oracle.response(2, zp, x, np.zeros_like(x), pl, th2, 0.5)
    H2 = oracle.unpack_hess(h2, 4)[0]
    H1 = oracle.unpack_hess(h1, 2)[0]
    np.testing.assert_allclose(R1, R2, rtol=1e-15)
    np.testing.assert_allclose(g1[0], g2[0, [0, 2]], rtol=1e-14)
    np.testing.assert_allclose(H1, H2[np.ix_([0, 2], [0, 2])], rtol=1e-14)


def test_empty_event():
    z = np.array([1.0], np.float32)
    R, g, h = oracle.response(2, z, np.zeros(0, np.float32), np.zeros(0, np.float32),
                              np.zeros(0, np.int32), [0, 0, 0, 0], 1.0)
    assert R[0] == 0.0 and np.all(g == 0) and np.all(h == 0)
