"""The FP32 tolerance used by the GPU parity tests is a forward error bound, not
a fitted number: here an FP32 emulation of the response arithmetic (the line's
position x0 + t z on the plane split exactly into s + l, residual (x - s) - l;
exp of the rounded argument; FP32 running sums) must stay inside that bound
relative to the FP64 oracle, while coarser arithmetic must not: the product t*z
rounded on its own, or the split compiled with its sums fused into fmas."""
import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events

from gpu_util import assert_response_bounded, fp32_error_model

f32 = np.float32


def _fma(a, b, c):
    """fl32(a b + c): the product of two floats is exact in FP64."""
    return (np.float64(a) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def _split(o, t, z, contracted=False):
    """s + l = o + t z: exact product error by fma, exact sum error by two-sum.
    contracted: the same source compiled with every product-plus-sum fused into
    an fma (s = fma(t, z, o), s - p as fma(-t, z, s), p - (s - bb) as
    fma(t, z, -(s - bb))), which leaves s + l wrong by up to an ulp of s."""
    p = (t * z).astype(np.float32)
    pe = _fma(t, z, -p)
    if contracted:
        s = _fma(t, z, o)
        bb = _fma(-t, z, s)
        se = ((o - bb).astype(np.float32) + _fma(t, z, -(s - bb).astype(np.float32))).astype(np.float32)
        return s, (pe + se).astype(np.float32)
    s = (p + o).astype(np.float32)
    bb = (s - p).astype(np.float32)
    se = ((p - (s - bb)).astype(np.float32) + (o - bb).astype(np.float32)).astype(np.float32)
    return s, (pe + se).astype(np.float32)


def _emulate(D, zp, x, y, pl, theta, sigma, mode="split"):
    """FP32 evaluation of R, g, packed H with plain per-hit accumulation."""
    z = zp.astype(np.float32)[pl]
    th = theta.astype(np.float32)
    npar = 2 * D
    nc = f32(-1.4426950408889634) / f32(f32(sigma) * f32(sigma))
    R = np.zeros(len(th), np.float32)
    G = np.zeros((len(th), npar), np.float32)
    H = np.zeros((len(th), npar * (npar + 1) // 2), np.float32)
    for i, t in enumerate(th):
        def resid(h, o, t):
            if mode == "unfused":  # t*z rounded on its own
                u = (h - (t * z).astype(np.float32)).astype(np.float32)
                return (u - o).astype(np.float32)
            sp, lp = _split(o, t, z, contracted=(mode == "contracted"))
            return ((h - sp).astype(np.float32) - lp).astype(np.float32)
        if D == 2:
            rx, ry = resid(x, t[0], t[2]), resid(y, t[1], t[3])
            d2 = (rx * rx + ry * ry).astype(np.float32)
            v = [rx, ry, (rx * z).astype(np.float32), (ry * z).astype(np.float32)]
        else:
            r = resid(x, t[0], t[1])
            d2 = (r * r).astype(np.float32)
            v = [r, (r * z).astype(np.float32)]
        e = np.exp2((d2 * nc).astype(np.float32).astype(np.float64)).astype(np.float32)
        two = f32(2) / f32(f32(sigma) * f32(sigma))
        four = two * two
        R[i] = np.sum(e, dtype=np.float32)
        for a in range(npar):
            G[i, a] = two * np.sum((e * v[a]).astype(np.float32), dtype=np.float32)
        q = 0
        for a in range(npar):
            for b in range(a, npar):
                phi = 0.0
                if D == 2:
                    pa = [(1, 0), (0, 1), (z, 0), (0, z)]
                else:
                    pa = [(1,), (z,)]
                phi = sum(np.asarray(pa[a][c], np.float32) * np.asarray(pa[b][c], np.float32) for c in range(D))
                term = (four * (e * v[a] * v[b]).astype(np.float32) - two * (e * phi).astype(np.float32))
                H[i, q] = np.sum(term.astype(np.float32), dtype=np.float32)
                q += 1
    return R, G, H


def _case(D):
    if D == 2:
        cfg = events.load_config("c2")
        b = events.make_batch(cfg, 1)
        ev = b.event(0)
        rng = np.random.default_rng(0)
        th = np.concatenate([ev.truth[:40] + rng.normal(0, 0.02, (40, 4)) * [1, 1, 1e-4, 1e-4],
                             np.c_[np.zeros((40, 2)), rng.uniform(-0.3, 0.3, (40, 2))]])
        return b, ev, th.astype(np.float32).astype(np.float64), 0.03, 750.0
    cfg = events.load_config("c1")
    b = events.make_batch(cfg, 1)
    ev = b.event(0)
    rng = np.random.default_rng(1)
    th = np.c_[rng.uniform(-0.5, 0.5, 300), rng.uniform(-1, 1, 300)]
    return b, ev, th.astype(np.float32).astype(np.float64), 0.02, 8.0


def test_fp32_emulation_within_model_bound():
    for D in (1, 2):
        b, ev, th, sigma, zmax = _case(D)
        Rr, Gr, Hr = oracle.response(D, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
        R, G, H = _emulate(D, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
        model = fp32_error_model(D, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
        assert_response_bounded(R, Rr, G, Gr, H, Hr, model, ev.n_hits, sigma, zmax)


def test_split_is_exact_to_second_order():
    """s + l represents x0 + t z to ~u^2 of its size, on the c2 slope and plane
    ranges (|t z| up to 225 mm)."""
    rng = np.random.default_rng(3)
    t = rng.uniform(-0.3, 0.3, 100000).astype(np.float32)
    z = rng.uniform(20, 750, 100000).astype(np.float32)
    o = rng.normal(0, 0.1, 100000).astype(np.float32)
    s, l = _split(o, t, z)
    exact = o.astype(np.float64) + t.astype(np.float64) * z.astype(np.float64)
    err = np.abs(s.astype(np.float64) + l.astype(np.float64) - exact)
    assert np.all(err <= 2.0 ** -46 * (np.abs(exact) + np.abs(o)))
    s2, l2 = _split(o, t, z, contracted=True)
    err2 = np.abs(s2.astype(np.float64) + l2.astype(np.float64) - exact)
    assert err2.max() > 2.0 ** -30 * np.abs(exact).max()


@pytest.mark.parametrize("mode", ["unfused", "contracted"])
def test_model_rejects_coarser_residuals(mode):
    """Rounding t*z on its own (|t z| up to ~260 mm), or a split whose sums were
    fused into fmas (its error terms then miss an ulp of s), costs ~1e-5 mm per
    residual: the bound must flag both, so it is tight enough to see either."""
    b, ev, th, sigma, zmax = _case(2)
    Rr, Gr, Hr = oracle.response(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
    R, G, H = _emulate(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma, mode=mode)
    model = fp32_error_model(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
    try:
        assert_response_bounded(R, Rr, G, Gr, H, Hr, model, ev.n_hits, sigma, zmax)
    except AssertionError:
        return
    raise AssertionError("the error model accepted %s residuals" % mode)
