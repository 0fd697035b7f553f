"""Helpers shared by the GPU parity tests (comparison rules only)."""
import numpy as np

from oracle.evaluate import _dist, match_tracks

# scale floors for parameter parity: |dp| <= 1e-4 * max(|p|, s_p)
S_P = {2: np.array([0.05, 0.05, 0.01, 0.01]), 1: np.array([0.01, 0.01])}


FP32_TINY = 2.0 ** -126  # smallest normal FP32: the GPU's exp2 flushes smaller terms to zero
U32 = 2.0 ** -24          # FP32 unit roundoff


def fp32_error_model(D, plane_z, x, y, plane, theta, sigma, chunk=2048):
    """Forward error model of an FP32 evaluation of Eq. (1) and its derivatives.

    For every theta returns (E, S): E = (E_R, E_G, E_H) bounds the sum over hits of
    each term's absolute error and S = (S_R, S_G, S_H) sums the terms' absolute
    values.  The kernels form a residual as (x - s) - l, with s + l = x0 + t z
    split exactly once per plane: x - s is exact when x is within a factor 2 of
    s and otherwise rounds by u|x - s|, the subtraction of l rounds by u|r|, and
    l itself is rounded at u|l| <= 2u^2(|t z| + |x0|), so
    eps_r <= u(2|r| + 4u(|x| + |t z| + |x0|)); exp(-r^2/sigma^2) then carries a relative error
    2|r| eps_r / sigma^2 plus the rounding of its argument (~4u(1 + r^2/sigma^2));
    gradient and Hessian terms also carry eps_r through their residual factors.
    Summation adds ~sqrt(N) u of S (applied by assert_response_bounded)."""
    z = np.asarray(plane_z, np.float64)[np.asarray(plane)]
    x = np.asarray(x, np.float64)
    y = None if y is None else np.asarray(y, np.float64)
    theta = np.asarray(theta, np.float64).reshape(-1, 2 * D)
    n = theta.shape[0]
    npar = 2 * D
    ER = np.zeros(n)
    SR = np.zeros(n)
    SG = np.zeros((n, npar))
    SH = np.zeros((n, npar * (npar + 1) // 2))
    EG = np.zeros_like(SG)
    EH = np.zeros_like(SH)
    s2 = sigma * sigma
    for i0 in range(0, n, chunk):
        th = theta[i0:i0 + chunk]
        if D == 2:
            tzx = th[:, 2:3] * z[None, :]
            tzy = th[:, 3:4] * z[None, :]
            rx = x[None, :] - tzx - th[:, 0:1]
            ry = y[None, :] - tzy - th[:, 1:2]
            ex = U32 * (2 * np.abs(rx) + 4 * U32 * (np.abs(x)[None, :] + np.abs(tzx) + np.abs(th[:, 0:1])))
            ey = U32 * (2 * np.abs(ry) + 4 * U32 * (np.abs(y)[None, :] + np.abs(tzy) + np.abs(th[:, 1:2])))
            a = (rx ** 2 + ry ** 2) / s2
            rel = 2 * (np.abs(rx) * ex + np.abs(ry) * ey) / s2 + 4 * U32 * (1 + a)
            comps = [np.abs(rx), np.abs(ry), np.abs(rx) * z, np.abs(ry) * z]
            errs = [ex, ey, ex * z, ey * z]
            phi = [(1.0, 0.0), (0.0, 1.0), (z, 0.0), (0.0, z)]
        else:
            tz = th[:, 1:2] * z[None, :]
            r = x[None, :] - tz - th[:, 0:1]
            e_r = U32 * (2 * np.abs(r) + 4 * U32 * (np.abs(x)[None, :] + np.abs(tz) + np.abs(th[:, 0:1])))
            a = r ** 2 / s2
            rel = 2 * np.abs(r) * e_r / s2 + 4 * U32 * (1 + a)
            comps = [np.abs(r), np.abs(r) * z]
            errs = [e_r, e_r * z]
            phi = [(1.0,), (z,)]
        e = np.exp(-a)
        er = e * rel  # absolute error of each exponential
        ER[i0:i0 + chunk] = er.sum(axis=1)
        SR[i0:i0 + chunk] = e.sum(axis=1)
        for k in range(npar):
            # magnitude; error from the exponential and from the residual itself
            SG[i0:i0 + chunk, k] = (2 / s2) * (e * comps[k]).sum(axis=1)
            EG[i0:i0 + chunk, k] = (2 / s2) * (er * comps[k] + e * errs[k]).sum(axis=1)
        q = 0
        for k in range(npar):
            for m in range(k, npar):
                pp = sum(np.asarray(phi[k][c]) * np.asarray(phi[m][c]) for c in range(D))
                mag = (4 / s2 ** 2) * comps[k] * comps[m] + (2 / s2) * np.abs(pp)
                SH[i0:i0 + chunk, q] = (e * mag).sum(axis=1)
                EH[i0:i0 + chunk, q] = (er * mag + (4 / s2 ** 2) * e * (comps[k] * errs[m] + comps[m] * errs[k])).sum(axis=1)
                q += 1
    return (ER, EG, EH), (SR, SG, SH)


def assert_response_bounded(R_gpu, R_ref, G_gpu, G_ref, H_gpu, H_ref, model, n_hits, sigma, z_max):
    """R within 1e-5 relative, G and H within 1e-4 relative, each widened by the FP32
    forward error bound of fp32_error_model (3x margin) and the underflow bound."""
    (ER, EG, EH), (SR, SG, SH) = model
    zm = max(1.0, z_max)
    summ = 4 * np.sqrt(max(n_hits, 1)) * U32
    uf = {"R": n_hits * FP32_TINY, "grad": n_hits * FP32_TINY * 20 * zm / sigma,
          "hess": n_hits * FP32_TINY * 400 * zm ** 2 / sigma ** 2}
    R_gpu = np.asarray(R_gpu, np.float64)
    tol = 1e-5 * np.abs(R_ref) + 3 * ER + summ * SR + uf["R"]
    bad = np.abs(R_gpu - R_ref) > tol
    assert not bad.any(), "R mismatch at %s: gpu %s ref %s" % (np.nonzero(bad)[0][:5], R_gpu[bad][:5], R_ref[bad][:5])
    for Gg, Gr, S, E, name, rt in ((G_gpu, G_ref, SG, EG, "grad", 1e-4), (H_gpu, H_ref, SH, EH, "hess", 1e-4)):
        if Gg is None:
            continue
        Gg = np.asarray(Gg, np.float64)
        tol = rt * np.abs(Gr) + 3 * E + summ * S + uf[name]
        bad = np.abs(Gg - Gr) > tol
        assert not bad.any(), "%s mismatch rows %s" % (name, np.nonzero(bad.any(axis=1))[0][:5])


def assert_response_close(R_gpu, R_ref, G_gpu=None, G_ref=None, H_gpu=None, H_ref=None,
                          n_hits=1, sigma=1.0, z_max=1.0):
    """R within 1e-5 relative; gradient and Hessian entries within 1e-4 relative
    with a floor of 1e-6 of the row's largest entry.  Every comparison also allows
    the FP32 underflow bound: each of the n_hits terms below 2^-126 is flushed to
    zero, and such a term sits at |r| <= sigma*sqrt(126 ln 2) < 10 sigma, so it
    contributes at most 2^-126 to R, 20 z_max/sigma * 2^-126 to a gradient entry
    and 400 max(1, z_max)^2/sigma^2 * 2^-126 to a Hessian entry."""
    R_gpu = np.asarray(R_gpu, np.float64)
    zm = max(1.0, z_max)
    uf = {"R": n_hits * FP32_TINY, "grad": n_hits * FP32_TINY * 20 * zm / sigma,
          "hess": n_hits * FP32_TINY * 400 * zm ** 2 / sigma ** 2}
    err = np.abs(R_gpu - R_ref)
    bad = err > 1e-5 * np.abs(R_ref) + uf["R"]
    assert not bad.any(), "R mismatch at %s: gpu %s ref %s" % (np.nonzero(bad)[0][:5], R_gpu[bad][:5], R_ref[bad][:5])
    for Gg, Gr, name in ((G_gpu, G_ref, "grad"), (H_gpu, H_ref, "hess")):
        if Gg is None:
            continue
        Gg = np.asarray(Gg, np.float64)
        row_max = np.abs(Gr).max(axis=1, keepdims=True)
        tol = 1e-4 * np.abs(Gr) + 1e-6 * row_max + uf[name]
        bad = np.abs(Gg - Gr) > tol
        assert not bad.any(), "%s mismatch rows %s" % (name, np.nonzero(bad.any(axis=1))[0][:5])


def assert_tracks_match(D, gpu_theta, gpu_R, ref_theta, ref_R, d_merge, z0, z1):
    """Track sets identical after matching within d_merge; parameters within 1e-4
    relative (scale floors S_P); R within 1e-5 relative.  Returns the per-track
    parameter error |dp| / max(|p|, s_p) (max over components)."""
    gpu_theta = np.asarray(gpu_theta, np.float64).reshape(-1, 2 * D)
    ref_theta = np.asarray(ref_theta, np.float64).reshape(-1, 2 * D)
    assert gpu_theta.shape[0] == ref_theta.shape[0], \
        "track counts differ: gpu %d oracle %d" % (gpu_theta.shape[0], ref_theta.shape[0])
    if ref_theta.shape[0] == 0:
        return np.zeros(0)
    f2t, t2f, d = match_tracks(D, gpu_theta, ref_theta, d_merge, z0, z1)
    assert np.all(f2t >= 0) and np.all(t2f >= 0), "unmatched tracks: gpu %s oracle %s" % (
        np.nonzero(f2t < 0)[0], np.nonzero(t2f < 0)[0])
    g = gpu_theta[t2f]
    rel = np.abs(g - ref_theta) / np.maximum(np.abs(ref_theta), S_P[D])
    assert rel.max() <= 1e-4, "parameter error %g" % rel.max()
    Rg = np.asarray(gpu_R, np.float64)[t2f]
    np.testing.assert_allclose(Rg, ref_R, rtol=1e-5)
    # the FP32-vs-FP64 error of this track set (shown with pytest -s)
    absd = np.abs(g - ref_theta).max(axis=0)
    print("    %d tracks: max |dp|/max(|p|, s_p) %.2e, max |dp| per component %s, max |dR|/R %.2e" % (
        len(ref_theta), rel.max(), " ".join("%.1e" % v for v in absd),
        float(np.max(np.abs(Rg - ref_R) / np.maximum(np.abs(ref_R), 1e-30)))), flush=True)
    return rel.max(axis=1)


def event_tracks(res, e, D):
    a, b = int(res["track_offsets"][e]), int(res["track_offsets"][e + 1])
    t = res["tracks"][a:b]
    return t["theta"][:, :2 * D], t["R"]


def assert_tracks_match_up_to_convergence_flags(D, gpu, ref, e, d_merge, z0, z1, seed_tol=1e-6):
    """Track-set parity where a track may hang on a single seed (rules that bring
    few seeds to convergence): matched tracks as assert_tracks_match; a track on
    one side only is accepted when every seed that supports it (converged, within
    d_merge of it) ended at the same point on the other side (|dp| <= seed_tol
    relative, scale floors S_P), i.e. the two sides differ only in the
    convergence decision (last polish step against conv_tol), not in a
    trajectory.  gpu/ref: result dicts with per-seed arrays (global seed order)
    and their seed offsets; returns (matched, boundary-only) counts."""
    so_g, so_r = gpu["seed_offsets"], ref["seed_offsets"]
    sg = slice(int(so_g[e]), int(so_g[e + 1]))
    sr = slice(int(so_r[e]), int(so_r[e + 1]))
    th_g, th_r = np.asarray(gpu["seed_theta"][sg], np.float64), np.asarray(ref["seed_theta"][sr], np.float64)
    assert th_g.shape == th_r.shape
    seed_rel = (np.abs(th_g - th_r) / np.maximum(np.abs(th_r), S_P[D])).max(axis=1) if len(th_r) else np.zeros(0)
    tg, Rg = gpu["tracks_theta"][e], gpu["tracks_R"][e]
    tr, Rr = ref["tracks_theta"][e], ref["tracks_R"][e]
    f2t, t2f, _ = match_tracks(D, tg, tr, d_merge, z0, z1)
    m = t2f >= 0
    if m.any():
        rel = np.abs(tg[t2f[m]] - tr[m]) / np.maximum(np.abs(tr[m]), S_P[D])
        assert rel.max() <= 1e-4, "parameter error %g" % rel.max()
        np.testing.assert_allclose(Rg[t2f[m]], Rr[m], rtol=1e-5)
    boundary = 0
    for side_tracks, miss, th_side, fl_side in ((tr, np.nonzero(t2f < 0)[0], th_r, ref["seed_flags"][sr]),
                                                (tg, np.nonzero(f2t < 0)[0], th_g, gpu["seed_flags"][sg])):
        for k in miss:
            dd = _dist(D, th_side, side_tracks[k][None, :], z0, z1)[:, 0]
            sup = np.nonzero((dd <= d_merge) & ((np.asarray(fl_side) & 1) > 0))[0]
            assert len(sup) > 0
            assert np.all(seed_rel[sup] <= seed_tol), \
                "track on one side only and its seeds' trajectories differ (%s)" % seed_rel[sup]
            boundary += 1
    return int(m.sum()), boundary
