"""The FP32 tolerance used by the GPU parity tests is a forward error bound, not
a fitted number: here an FP32 emulation of the response arithmetic (residual
by one rounding of x - t z, then minus x0; exp of the rounded argument; FP32
running sums) must stay inside that bound relative to the FP64 oracle, while a
deliberately coarser arithmetic (the product t*z rounded on its own) must not."""
import numpy as np

import oracle
from paper_1709_08610_amd import events

from gpu_util import assert_response_bounded, fp32_error_model

f32 = np.float32


def _emulate(D, zp, x, y, pl, theta, sigma, fused=True):
    """FP32 evaluation of R, g, packed H with plain per-hit accumulation."""
    z = zp.astype(np.float32)[pl]
    th = theta.astype(np.float32)
    npar = 2 * D
    nc = f32(-1.4426950408889634) / f32(f32(sigma) * f32(sigma))
    R = np.zeros(len(th), np.float32)
    G = np.zeros((len(th), npar), np.float32)
    H = np.zeros((len(th), npar * (npar + 1) // 2), np.float32)
    for i, t in enumerate(th):
        def resid(h, o, s):
            if fused:  # one rounding of h - s*z (exact product in FP64), then - o
                u = (h.astype(np.float64) - s.astype(np.float64) * z.astype(np.float64)).astype(np.float32)
            else:
                u = (h - (s * z).astype(np.float32)).astype(np.float32)
            return (u - o).astype(np.float32)
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


def test_model_rejects_unfused_residuals():
    """Rounding t*z on its own (|t z| up to ~260 mm) costs ~1e-5 mm per residual:
    the bound must flag it, so it is tight enough to see that mistake."""
    b, ev, th, sigma, zmax = _case(2)
    Rr, Gr, Hr = oracle.response(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
    R, G, H = _emulate(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma, fused=False)
    model = fp32_error_model(2, b.plane_z, ev.x, ev.y, ev.plane, th, sigma)
    try:
        assert_response_bounded(R, Rr, G, Gr, H, Hr, model, ev.n_hits, sigma, zmax)
    except AssertionError:
        return
    raise AssertionError("the error model accepted unfused residuals")
