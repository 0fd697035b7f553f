"""FP64 CPU oracle: Python side (ctypes marshalling of oracle.c, plus the
evaluation steps that are plain definitions).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the library or its binding.  It
shares no code with the HIP path; the only common input is the seeded event
generator, which holds none of the method's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# a sanitizer build of the same source (build_sanitized) may stand in
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")
_lib = None

CONVERGED, STALLED, NOT_PD, NEGCURV = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP, no fast-math, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("n_sigma", ctypes.c_int32), ("sigma", ctypes.POINTER(ctypes.c_float)),
                ("sigma_final", ctypes.c_float), ("n_final_steps", ctypes.c_int32),
                ("n_polish", ctypes.c_int32), ("ls_trials", ctypes.c_int32),
                ("armijo_c1", ctypes.c_float), ("step_cap_sigmas", ctypes.c_float),
                ("small_step_sigmas", ctypes.c_float), ("n_slope_steps", ctypes.c_int32),
                ("conv_tol", ctypes.c_float),
                ("R0", ctypes.c_float), ("d_merge", ctypes.c_float),
                ("lattice_n", ctypes.c_int32 * 2), ("lattice_lo", ctypes.c_float * 2),
                ("lattice_hi", ctypes.c_float * 2), ("update", ctypes.c_int32)]


def build_sanitized(path: str) -> str:
    """oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer (a CPU
    check of the checker; load it by setting ORACLE_LIB=path with the ASan
    runtime preloaded)."""
    src = os.path.join(_HERE, "oracle.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-Wall", "-o", path, src, "-lm"])
    return path


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_OVERRIDE or _LIB_PATH)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_response.argtypes = [ctypes.c_int, ctypes.c_int, P, I64, P, P, P, I64, P, D, P, P, P]
        lib.oracle_response.restype = None
        lib.oracle_newton_cg.argtypes = [ctypes.c_int, P, P, P, D, D, P, P, P]
        lib.oracle_newton_cg.restype = None
        lib.oracle_merge.argtypes = [ctypes.c_int, I64, P, P, P, D, D, D, D, P, P]
        lib.oracle_merge.restype = I64
        lib.oracle_find_tracks.argtypes = [ctypes.c_int, ctypes.c_int, P, I64, P, P, P, P,
                                           ctypes.POINTER(Params), P, P, P, P, P, P, P, P, P, P, P,
                                           ctypes.c_int]
        lib.oracle_find_tracks.restype = ctypes.c_int
        lib.oracle_polish.argtypes = [ctypes.c_int, ctypes.c_int, P, I64, P, P, P, I64, P, D,
                                      ctypes.c_int, P, P, P]
        lib.oracle_polish.restype = None
        lib.oracle_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(Params), P]
        lib.oracle_lattice.restype = None
        lib.oracle_grid_search.argtypes = [ctypes.c_int, ctypes.c_int, P, I64, P, P, P, ctypes.POINTER(Params),
                                           D, D, P, I64, P, P, P, P, ctypes.c_int]
        lib.oracle_grid_search.restype = I64
        lib.oracle_bfgs_update.argtypes = [ctypes.c_int, P, P, P]
        lib.oracle_bfgs_update.restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


UPDATE_RULES = {"newton": 0, "gradient": 1, "bfgs": 2}


def make_params(p: dict):
    """ctypes Params from a config's "params" dict; keeps the sigma array alive."""
    sig = np.ascontiguousarray(p["sigma"], dtype=np.float32)
    P = Params()
    P.n_sigma = len(sig)
    P.sigma = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    P.sigma_final = p["sigma_final"]
    P.n_final_steps = p["n_final_steps"]
    P.n_polish = p["n_polish"]
    P.ls_trials = p["ls_trials"]
    P.armijo_c1 = p["armijo_c1"]
    P.step_cap_sigmas = p["step_cap_sigmas"]
    P.small_step_sigmas = p["small_step_sigmas"]
    P.n_slope_steps = p.get("n_slope_steps", 0)
    P.conv_tol = p["conv_tol"]
    P.R0 = p["R0"]
    P.d_merge = p["d_merge"]
    P.lattice_n[:] = list(p["lattice_n"])
    P.lattice_lo[:] = list(p["lattice_lo"])
    P.lattice_hi[:] = list(p["lattice_hi"])
    P.update = UPDATE_RULES[p.get("update", "newton")]
    return P, sig


def response(meas_dim, plane_z, x, y, plane, theta, sigma, want_derivs=True):
    """Eq. (1) and its derivatives at each row of theta (one event, FP64).

    Returns (R [n], grad [n, n_par], hess [n, n_par*(n_par+1)/2] packed upper)."""
    lib = _load()
    D = int(meas_dim)
    npar = 2 * D
    z = _c(plane_z, np.float32)
    x = _c(x, np.float32)
    y = _c(y, np.float32) if D == 2 else None
    plane = _c(plane, np.int32)
    th = _c(np.atleast_2d(theta), np.float64)
    n = th.shape[0]
    R = np.zeros(n)
    g = np.zeros((n, npar)) if want_derivs else None
    h = np.zeros((n, npar * (npar + 1) // 2)) if want_derivs else None
    lib.oracle_response(D, z.shape[0], _p(z), x.shape[0], _p(x), _p(y), _p(plane), n, _p(th),
                        float(sigma), _p(R), _p(g), _p(h))
    return R, g, h


def unpack_hess(h, npar):
    """Packed upper row-major -> full symmetric matrices [n, npar, npar]."""
    h = np.atleast_2d(h)
    out = np.zeros((h.shape[0], npar, npar))
    q = 0
    for a in range(npar):
        for b in range(a, npar):
            out[:, a, b] = h[:, q]
            out[:, b, a] = h[:, q]
            q += 1
    return out


def newton_cg(g, H, dscale, sigma, cap):
    """Truncated-Newton direction (see oracle.c); returns (p, |p~|, negcurv)."""
    lib = _load()
    g = _c(g, np.float64)
    npar = g.shape[0]
    H = _c(np.asarray(H).reshape(npar, npar), np.float64)
    ds = _c(dscale, np.float64)
    p = np.zeros(npar)
    pn = ctypes.c_double()
    neg = ctypes.c_int()
    lib.oracle_newton_cg(npar, _p(g), _p(H), _p(ds), float(sigma), float(cap), _p(p),
                         ctypes.byref(pn), ctypes.byref(neg))
    return p, pn.value, bool(neg.value)


def merge(meas_dim, theta, R, flags, R0, d_merge, z_first, z_last):
    """Cluster + select for one event; returns (leader seed indices, members)."""
    lib = _load()
    th = _c(theta, np.float64)
    R = _c(R, np.float64)
    fl = _c(flags, np.int32)
    n = R.shape[0]
    ld = np.zeros(max(n, 1), np.int64)
    mem = np.zeros(max(n, 1), np.int32)
    nl = lib.oracle_merge(int(meas_dim), n, _p(th), _p(R), _p(fl), float(R0), float(d_merge),
                          float(z_first), float(z_last), _p(ld), _p(mem))
    return ld[:nl].copy(), mem[:nl].copy()


def lattice(meas_dim, params: dict):
    lib = _load()
    P, keep = make_params(params)
    n = params["lattice_n"][0] * params["lattice_n"][1]
    out = np.zeros((n, 2 * meas_dim))
    lib.oracle_lattice(int(meas_dim), ctypes.byref(P), _p(out))
    return out


def find_tracks(batch, params: dict, seeds=None, seed_offsets=None, n_threads=0):
    """Algorithm 1 over a generator Batch (or anything with the same fields).

    Returns a dict with per-event track lists and per-seed results."""
    lib = _load()
    D = int(batch.meas_dim)
    npar = 2 * D
    P, keep = make_params(params)
    z = _c(batch.plane_z, np.float32)
    off = _c(batch.event_offsets, np.int64)
    x = _c(batch.x, np.float32)
    y = _c(batch.y, np.float32) if D == 2 else None
    pl = _c(batch.plane, np.int32)
    E = off.shape[0] - 1
    if seeds is not None:
        seeds = _c(seeds, np.float64).reshape(-1, npar)
        seed_offsets = _c(seed_offsets, np.int64)
        ns = int(seed_offsets[-1])
    else:
        ns = E * params["lattice_n"][0] * params["lattice_n"][1]
    st = np.zeros((max(ns, 1), npar))
    sR = np.zeros(max(ns, 1))
    sf = np.zeros(max(ns, 1), np.int32)
    snr = np.zeros(max(ns, 1), np.int32)
    tt = np.zeros((max(ns, 1), npar))
    tR = np.zeros(max(ns, 1))
    tm = np.zeros(max(ns, 1), np.int32)
    tsd = np.zeros(max(ns, 1), np.int64)
    toff = np.zeros(E + 1, np.int64)
    rc = lib.oracle_find_tracks(D, z.shape[0], _p(z), E, _p(off), _p(x), _p(y), _p(pl),
                                ctypes.byref(P), _p(seeds), _p(seed_offsets), _p(st), _p(sR),
                                _p(sf), _p(snr), _p(tt), _p(tR), _p(tm), _p(tsd), _p(toff),
                                int(n_threads))
    if rc != 0:
        raise RuntimeError("oracle_find_tracks failed (%d)" % rc)
    nt = int(toff[-1])
    return dict(track_offsets=toff, theta=tt[:nt], R=tR[:nt], members=tm[:nt], seed=tsd[:nt],
                seed_theta=st[:ns], seed_R=sR[:ns], seed_flags=sf[:ns], seed_nreval=snr[:ns])


def polish(meas_dim, plane_z, x, y, plane, theta, sigma, n_iter):
    lib = _load()
    D = int(meas_dim)
    z = _c(plane_z, np.float32)
    x = _c(x, np.float32)
    y = _c(y, np.float32) if D == 2 else None
    pl = _c(plane, np.int32)
    th = np.array(np.atleast_2d(theta), dtype=np.float64, copy=True)
    n = th.shape[0]
    R = np.zeros(n)
    st = np.zeros(n)
    pd = np.zeros(n, np.int32)
    lib.oracle_polish(D, z.shape[0], _p(z), x.shape[0], _p(x), _p(y), _p(pl), n, _p(th),
                      float(sigma), int(n_iter), _p(R), _p(st), _p(pd))
    return th, R, st, pd.astype(bool)


def bfgs_update(B, s, y):
    """The oracle's BFGS inverse-Hessian update (returns a new matrix)."""
    lib = _load()
    Bn = np.array(B, dtype=np.float64, copy=True)
    n = Bn.shape[0]
    lib.oracle_bfgs_update(n, _p(Bn), _p(np.ascontiguousarray(s, np.float64)), _p(np.ascontiguousarray(y, np.float64)))
    return Bn


def grid_search(meas_dim, plane_z, x, y, plane, grid: dict, n_threads=0, want_grid=True):
    """Grid-search Artificial Retina on ONE event (Section 2).  grid: n, lo, hi
    (the lattice box, as the seed lattice), sigma, R0.  Returns dict(R_grid
    [n0, n1] or None, cell [k], theta [k, n_par], R [k], members [k]), peaks in
    cell order."""
    lib = _load()
    D = int(meas_dim)
    P = Params()
    P.lattice_n[:] = list(grid["n"])
    P.lattice_lo[:] = list(grid["lo"])
    P.lattice_hi[:] = list(grid["hi"])
    z = _c(plane_z, np.float32)
    x = _c(x, np.float32)
    y = _c(y, np.float32) if D == 2 else None
    pl = _c(plane, np.int32)
    n0, n1 = int(grid["n"][0]), int(grid["n"][1])
    G = np.zeros((n0, n1)) if want_grid else None
    cap = n0 * n1
    cell = np.zeros(max(cap, 1), np.int64)
    th = np.zeros((max(cap, 1), 2 * D))
    R = np.zeros(max(cap, 1))
    mem = np.zeros(max(cap, 1), np.int32)
    k = lib.oracle_grid_search(D, z.shape[0], _p(z), x.shape[0], _p(x), _p(y), _p(pl), ctypes.byref(P),
                               float(grid["sigma"]), float(grid["R0"]), _p(G), cap, _p(cell), _p(th), _p(R),
                               _p(mem), int(n_threads))
    if k < 0:
        raise ValueError("oracle_grid_search: bad geometry")
    return dict(R_grid=G, cell=cell[:k].copy(), theta=th[:k].copy(), R=R[:k].copy(), members=mem[:k].copy())


from .evaluate import match_tracks, efficiency  # noqa: E402  (plain-definition evaluation)
