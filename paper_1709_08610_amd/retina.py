"""ctypes binding of libretina (include/retina.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
(host memory) or torch tensors on the GPU (device memory) into the C
structures and calls the entry point of the same name.  A missing or
unloadable libretina.so raises immediately: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libretina.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_CAPACITY, ERR_INTERNAL = 0, -1, -2, -3, -4, -6
MEM_HOST, MEM_DEVICE = 0, 1
WANT_R, WANT_GRAD, WANT_HESS = 1, 2, 4
SEED_LATTICE, SEED_EXPLICIT = 0, 1
CONVERGED, STALLED, NOT_PD, NEGCURV = 1, 2, 4, 8
MAX_PLANES, MAX_SIGMA = 64, 16


class RetinaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libretina error %d: %s" % (code, msg))
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [("meas_dim", ctypes.c_int32), ("n_planes", ctypes.c_int32),
                ("plane_z", ctypes.POINTER(ctypes.c_float))]


class Hits(ctypes.Structure):
    _fields_ = [("mem", ctypes.c_int32), ("n_events", ctypes.c_int64),
                ("event_offsets", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("plane", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("n_sigma", ctypes.c_int32), ("sigma", ctypes.POINTER(ctypes.c_float)),
                ("sigma_final", ctypes.c_float), ("n_final_steps", ctypes.c_int32),
                ("n_polish", ctypes.c_int32), ("ls_trials", ctypes.c_int32),
                ("armijo_c1", ctypes.c_float), ("step_cap_sigmas", ctypes.c_float),
                ("small_step_sigmas", ctypes.c_float), ("n_slope_steps", ctypes.c_int32),
                ("conv_tol", ctypes.c_float), ("R0", ctypes.c_float), ("d_merge", ctypes.c_float),
                ("seed_mode", ctypes.c_int32), ("lattice_n", ctypes.c_int32 * 2),
                ("lattice_lo", ctypes.c_float * 2), ("lattice_hi", ctypes.c_float * 2),
                ("seeds", ctypes.c_void_p), ("seed_offsets", ctypes.c_void_p), ("update", ctypes.c_int32),
                ("prune_u", ctypes.c_float)]


class Track(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double * 4), ("R", ctypes.c_float), ("n_members", ctypes.c_int32),
                ("seed_index", ctypes.c_int32), ("flags", ctypes.c_int32)]


TRACK_DTYPE = np.dtype([("theta", np.float64, (4,)), ("R", np.float32), ("n_members", np.int32),
                        ("seed_index", np.int32), ("flags", np.int32)])
assert TRACK_DTYPE.itemsize == ctypes.sizeof(Track) == 48


class Proposal(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("tau", ctypes.c_float), ("conf_min", ctypes.c_float),
                ("nms", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 2), ("lo", ctypes.c_float * 2), ("hi", ctypes.c_float * 2),
                ("sigma", ctypes.c_float), ("R0", ctypes.c_float)]


class SeedOut(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("R", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("n_reval", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


_lib = None

class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("ms_stage", ctypes.c_double), ("ms_plan", ctypes.c_double),
                ("ms_hot", ctypes.c_double), ("ms_merge", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("exec_pairs", ctypes.c_double), ("exec_rpairs", ctypes.c_double),
                ("ms_propose", ctypes.c_double)]


EXPORTS = ["retina_create", "retina_destroy", "retina_last_error", "retina_set_stream",
           "retina_set_max_device_bytes", "retina_set_tuning", "retina_get_tuning",
           "retina_set_profiling", "retina_get_profile", "retina_profile_reset",
           "retina_set_graphs", "retina_autotune", "retina_response", "retina_find_tracks",
           "retina_model_create", "retina_model_save", "retina_model_load", "retina_model_free",
           "retina_model_get_params", "retina_model_set_params", "retina_model_step",
           "retina_train_step", "retina_model_forward", "retina_propose_seeds",
           "retina_find_tracks_learned", "retina_grid_search", "retina_response_noalloc"]
UPDATE_RULES = {"newton": 0, "gradient": 1, "bfgs": 2}   # RETINA_UPDATE_*
MODEL_PARAMS = 186625
IMG = 128
SLOPE_LO, SLOPE_HI = -0.35, 0.35


def load(path: str = LIB_PATH):
    """Load libretina.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libretina.so is not built (%s); run __graft_entry__.build()" % path)
    # One HIP runtime per process: PyTorch resolves "libamdhip64.so" from its own
    # directory, libretina resolves "libamdhip64.so.7" (the same SONAME).  Loading
    # torch's copy first lets libretina bind to it; the other order would leave two
    # runtimes in the process and torch would see no GPU.
    try:
        import torch  # noqa: F401
        if torch.version.hip is not None:
            ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"),
                        mode=ctypes.RTLD_GLOBAL)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    V, P = ctypes.c_void_p, ctypes.c_void_p
    lib.retina_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.retina_create.restype = ctypes.c_int
    lib.retina_destroy.argtypes = [V]
    lib.retina_destroy.restype = None
    lib.retina_last_error.argtypes = [V]
    lib.retina_last_error.restype = ctypes.c_char_p
    lib.retina_set_stream.argtypes = [V, V]
    lib.retina_set_stream.restype = ctypes.c_int
    lib.retina_set_max_device_bytes.argtypes = [V, ctypes.c_int64]
    lib.retina_set_max_device_bytes.restype = ctypes.c_int
    I32 = ctypes.c_int32
    lib.retina_set_profiling.argtypes = [V, I32]
    lib.retina_set_profiling.restype = ctypes.c_int
    lib.retina_get_profile.argtypes = [V, ctypes.POINTER(Profile)]
    lib.retina_get_profile.restype = ctypes.c_int
    lib.retina_profile_reset.argtypes = [V]
    lib.retina_profile_reset.restype = ctypes.c_int
    I64, F = ctypes.c_int64, ctypes.c_float
    lib.retina_model_create.argtypes = [V, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]
    lib.retina_model_create.restype = ctypes.c_int
    lib.retina_model_save.argtypes = [V, ctypes.c_char_p]
    lib.retina_model_save.restype = ctypes.c_int
    lib.retina_model_load.argtypes = [V, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.retina_model_load.restype = ctypes.c_int
    lib.retina_model_free.argtypes = [V]
    lib.retina_model_free.restype = None
    lib.retina_model_get_params.argtypes = [V, P]
    lib.retina_model_get_params.restype = ctypes.c_int
    lib.retina_model_set_params.argtypes = [V, P]
    lib.retina_model_set_params.restype = ctypes.c_int
    lib.retina_model_step.argtypes = [V]
    lib.retina_model_step.restype = I64
    lib.retina_train_step.argtypes = [V, V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), P, P, F, F,
                                      ctypes.POINTER(F), P]
    lib.retina_train_step.restype = ctypes.c_int
    lib.retina_model_forward.argtypes = [V, V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), P, P]
    lib.retina_model_forward.restype = ctypes.c_int
    lib.retina_propose_seeds.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), V,
                                         ctypes.POINTER(Proposal), ctypes.POINTER(Params), P, I64, P, P, P]
    lib.retina_propose_seeds.restype = ctypes.c_int
    lib.retina_find_tracks_learned.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits),
                                               ctypes.POINTER(Params), V, ctypes.POINTER(Proposal), P, I64, P, P]
    lib.retina_find_tracks_learned.restype = ctypes.c_int
    lib.retina_set_graphs.argtypes = [V, I32]
    lib.retina_set_graphs.restype = ctypes.c_int
    lib.retina_autotune.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), ctypes.POINTER(Params),
                                    ctypes.c_char_p, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.retina_autotune.restype = ctypes.c_int
    lib.retina_set_tuning.argtypes = [V, I32, I32, I32, I32]
    lib.retina_set_tuning.restype = ctypes.c_int
    lib.retina_get_tuning.argtypes = [V, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.retina_get_tuning.restype = ctypes.c_int
    lib.retina_response.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), P, ctypes.c_int64,
                                    P, ctypes.c_float, ctypes.c_uint32, P, P, P]
    lib.retina_response.restype = ctypes.c_int
    lib.retina_response_noalloc.argtypes = lib.retina_response.argtypes
    lib.retina_response_noalloc.restype = ctypes.c_int
    lib.retina_find_tracks.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits),
                                       ctypes.POINTER(Params), P, ctypes.c_int64, P, P,
                                       ctypes.POINTER(SeedOut)]
    lib.retina_find_tracks.restype = ctypes.c_int
    lib.retina_grid_search.argtypes = [V, ctypes.POINTER(Geometry), ctypes.POINTER(Hits), ctypes.POINTER(Grid),
                                       P, P, ctypes.c_int64, P]
    lib.retina_grid_search.restype = ctypes.c_int
    _lib = lib
    return lib


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    if a is None:
        return None
    if _is_torch(a):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _mem_of(a):
    if _is_torch(a):
        if not a.is_cuda:
            raise TypeError("torch tensors must live on the GPU (use numpy for host memory)")
        return MEM_DEVICE
    return MEM_HOST


def _host(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _dev(a, dt):
    import torch
    if a is None:
        return None
    if a.dtype != dt or not a.is_contiguous():
        raise TypeError("device array must be a contiguous %s tensor" % dt)
    return a


class Context:
    """One libretina context (device pool + stream) on a gfx950 device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        rc = self.lib.retina_create(int(device), ctypes.byref(h))
        if rc != OK:
            raise RetinaError(rc, "retina_create(%d) failed: no usable gfx950 device" % device)
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.retina_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise RetinaError(rc, self.lib.retina_last_error(self.h).decode())

    def set_stream(self, stream_handle: Optional[int]):
        self._check(self.lib.retina_set_stream(self.h, ctypes.c_void_p(stream_handle or 0)))

    def set_max_device_bytes(self, n: int):
        self._check(self.lib.retina_set_max_device_bytes(self.h, int(n)))

    def retina_set_profiling(self, enable: bool):
        self._check(self.lib.retina_set_profiling(self.h, int(bool(enable))))

    def retina_get_profile(self) -> dict:
        p = Profile()
        self._check(self.lib.retina_get_profile(self.h, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    def retina_profile_reset(self):
        self._check(self.lib.retina_profile_reset(self.h))

    def retina_set_tuning(self, meas_dim: int, kernel: int, cand: int, tile_hits: int):
        self._check(self.lib.retina_set_tuning(self.h, meas_dim, kernel, cand, tile_hits))

    def retina_get_tuning(self, meas_dim: int, kernel: int):
        c, t, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.retina_get_tuning(self.h, meas_dim, kernel, ctypes.byref(c),
                                               ctypes.byref(t), ctypes.byref(g)))
        return dict(cand=c.value, tile_hits=t.value, grid=g.value)

    # ------------------------------------------------------------ marshalling
    @staticmethod
    def _geometry(meas_dim, plane_z):
        z = np.ascontiguousarray(plane_z, dtype=np.float32)
        g = Geometry(int(meas_dim), int(z.shape[0]), z.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        return g, z

    def _hits(self, meas_dim, event_offsets, x, y, plane):
        mem = _mem_of(x)
        if mem == MEM_HOST:
            off = _host(event_offsets, np.int64)
            x = _host(x, np.float32)
            y = _host(y, np.float32) if meas_dim == 2 else None
            plane = _host(plane, np.int32)
        else:
            import torch
            off = _dev(event_offsets, torch.int64)
            x = _dev(x, torch.float32)
            y = _dev(y, torch.float32) if meas_dim == 2 else None
            plane = _dev(plane, torch.int32)
        hits = Hits(mem, int(off.shape[0]) - 1, _ptr(off), _ptr(x), _ptr(y), _ptr(plane))
        return hits, (off, x, y, plane), mem

    @staticmethod
    def _params(params, seeds, seed_offsets, mem, npar, E):
        sig = np.ascontiguousarray(params["sigma"], dtype=np.float32)
        P = Params()
        P.n_sigma = len(sig)
        P.sigma = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        for k in ("sigma_final", "n_final_steps", "n_polish", "ls_trials", "armijo_c1",
                  "step_cap_sigmas", "small_step_sigmas", "conv_tol", "R0", "d_merge"):
            setattr(P, k, params[k])
        P.n_slope_steps = params.get("n_slope_steps", 0)
        P.lattice_n[:] = list(params["lattice_n"])
        P.lattice_lo[:] = list(params["lattice_lo"])
        P.lattice_hi[:] = list(params["lattice_hi"])
        P.update = UPDATE_RULES[params.get("update", "newton")]
        P.prune_u = float(params.get("prune_u", 0.0))
        if seeds is not None:
            P.seed_mode = SEED_EXPLICIT
            if mem == MEM_HOST:
                seeds = _host(seeds, np.float64).reshape(-1, npar)
                seed_offsets = _host(seed_offsets, np.int64)
                n_seeds = int(seed_offsets[-1])
            else:
                import torch
                seeds = _dev(seeds, torch.float64)
                seed_offsets = _dev(seed_offsets, torch.int64)
                n_seeds = int(seed_offsets[-1].item())
            P.seeds = _ptr(seeds)
            P.seed_offsets = _ptr(seed_offsets)
        else:
            P.seed_mode = SEED_LATTICE
            n_seeds = E * params["lattice_n"][0] * params["lattice_n"][1]
        return P, (sig, seeds, seed_offsets), n_seeds

    def retina_set_graphs(self, enable: bool):
        self._check(self.lib.retina_set_graphs(self.h, int(bool(enable))))

    def retina_autotune(self, meas_dim, plane_z, event_offsets, x, y, plane, params: dict,
                        cache_path: Optional[str] = None, seeds=None, seed_offsets=None):
        """Time the ascent launch shapes on this sample batch and install the fastest."""
        g, zkeep = self._geometry(meas_dim, plane_z)
        hits, keep, mem = self._hits(meas_dim, event_offsets, x, y, plane)
        P, pkeep, _ = self._params(params, seeds, seed_offsets, mem, 2 * meas_dim, hits.n_events)
        if mem == MEM_DEVICE:
            import torch
            self.set_stream(torch.cuda.current_stream(x.device).cuda_stream)
        c, t = ctypes.c_int32(), ctypes.c_int32()
        rc = self.lib.retina_autotune(self.h, ctypes.byref(g), ctypes.byref(hits), ctypes.byref(P),
                                      cache_path.encode() if cache_path else None, ctypes.byref(c), ctypes.byref(t))
        self._check(rc)
        return dict(cand=c.value, tile_hits=t.value)

    # ------------------------------------------------------------- entries
    def retina_response(self, meas_dim, plane_z, event_offsets, x, y, plane, theta,
                        theta_offsets=None, sigma=1.0, want=WANT_R | WANT_GRAD | WANT_HESS):
        """Eq. (1) (+ gradient, packed Hessian) at each row of theta.
        Returns (R, grad, hess) in the memory space of the inputs."""
        return self._response(self.lib.retina_response, meas_dim, plane_z, event_offsets, x, y, plane, theta,
                              theta_offsets, sigma, want)

    def retina_response_noalloc(self, meas_dim, plane_z, event_offsets, x, y, plane, theta,
                                theta_offsets=None, sigma=1.0, want=WANT_R | WANT_GRAD | WANT_HESS,
                                out=None):
        """retina_response on the library's fixed device workspace (device
        memory only; the library allocates nothing).  `out` = (R, grad, hess)
        preallocated device tensors, else they are created here."""
        return self._response(self.lib.retina_response_noalloc, meas_dim, plane_z, event_offsets, x, y, plane,
                              theta, theta_offsets, sigma, want, out)

    def _response(self, fn, meas_dim, plane_z, event_offsets, x, y, plane, theta, theta_offsets, sigma, want,
                  out=None):
        g, zkeep = self._geometry(meas_dim, plane_z)
        hits, keep, mem = self._hits(meas_dim, event_offsets, x, y, plane)
        npar = 2 * meas_dim
        nh = npar * (npar + 1) // 2
        if mem == MEM_HOST:
            th = _host(theta, np.float32).reshape(-1, npar)
            to = _host(theta_offsets, np.int64) if theta_offsets is not None else None
            n = th.shape[0]
            R = np.zeros(n, np.float32)
            G = np.zeros((n, npar), np.float32) if want & WANT_GRAD else None
            H = np.zeros((n, nh), np.float32) if want & WANT_HESS else None
        else:
            import torch
            th = _dev(theta, torch.float32)
            to = _dev(theta_offsets, torch.int64) if theta_offsets is not None else None
            n = th.numel() // npar
            if out is not None:
                R, G, H = out
                R = _dev(R, torch.float32)
                G = _dev(G, torch.float32) if want & WANT_GRAD else None
                H = _dev(H, torch.float32) if want & WANT_HESS else None
                if R.numel() < n or (G is not None and G.numel() < n * npar) or (H is not None and H.numel() < n * nh):
                    raise ValueError("output tensors are smaller than n_theta results")
            else:
                R = torch.zeros(n, dtype=torch.float32, device=th.device)
                G = torch.zeros((n, npar), dtype=torch.float32, device=th.device) if want & WANT_GRAD else None
                H = torch.zeros((n, nh), dtype=torch.float32, device=th.device) if want & WANT_HESS else None
            self.set_stream(torch.cuda.current_stream(th.device).cuda_stream)
        rc = fn(self.h, ctypes.byref(g), ctypes.byref(hits), _ptr(th), int(n),
                _ptr(to), float(sigma), int(want), _ptr(R), _ptr(G), _ptr(H))
        self._check(rc)
        return R, G, H

    def retina_find_tracks(self, meas_dim, plane_z, event_offsets, x, y, plane, params: dict,
                           seeds=None, seed_offsets=None, capacity=None, want_seeds=False):
        """Algorithm 1 over the batch.  Returns dict(tracks (structured numpy
        array or uint8 tensor view), track_offsets, event_flags, seeds...)."""
        g, zkeep = self._geometry(meas_dim, plane_z)
        hits, keep, mem = self._hits(meas_dim, event_offsets, x, y, plane)
        npar = 2 * meas_dim
        E = hits.n_events
        P, pkeep, n_seeds = self._params(params, seeds, seed_offsets, mem, npar, E)
        cap = n_seeds if capacity is None else int(capacity)
        if mem == MEM_HOST:
            tracks = np.zeros(max(cap, 1), TRACK_DTYPE)
            toff = np.zeros(E + 1, np.int64)
            evf = np.zeros(max(E, 1), np.int32)
            so = None
            if want_seeds:
                st = np.zeros((max(n_seeds, 1), npar))
                sR = np.zeros(max(n_seeds, 1), np.float32)
                sf = np.zeros(max(n_seeds, 1), np.int32)
                snr = np.zeros(max(n_seeds, 1), np.int32)
        else:
            import torch
            dev = x.device
            self.set_stream(torch.cuda.current_stream(dev).cuda_stream)
            tracks = torch.empty(max(cap, 1) * 48, dtype=torch.uint8, device=dev)  # records [0, offsets[-1]) written
            toff = torch.zeros(E + 1, dtype=torch.int64, device=dev)
            evf = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
            if want_seeds:
                st = torch.zeros((max(n_seeds, 1), npar), dtype=torch.float64, device=dev)
                sR = torch.zeros(max(n_seeds, 1), dtype=torch.float32, device=dev)
                sf = torch.zeros(max(n_seeds, 1), dtype=torch.int32, device=dev)
                snr = torch.zeros(max(n_seeds, 1), dtype=torch.int32, device=dev)
        so_struct = SeedOut(_ptr(st), _ptr(sR), _ptr(sf), _ptr(snr), n_seeds) if want_seeds else None
        rc = self.lib.retina_find_tracks(self.h, ctypes.byref(g), ctypes.byref(hits), ctypes.byref(P),
                                         _ptr(tracks), cap, _ptr(toff), _ptr(evf),
                                         ctypes.byref(so_struct) if so_struct is not None else None)
        if rc == ERR_CAPACITY:
            need = int(toff[-1]) if mem == MEM_HOST else int(toff[-1].item())
            err = RetinaError(rc, self.lib.retina_last_error(self.h).decode())
            err.required = need
            raise err
        self._check(rc)
        out = dict(track_offsets=toff, event_flags=evf[:E])
        if mem == MEM_HOST:
            out["tracks"] = tracks[:int(toff[-1])]
        else:
            out["tracks_bytes"] = tracks
        if want_seeds:
            out.update(seed_theta=st[:n_seeds], seed_R=sR[:n_seeds], seed_flags=sf[:n_seeds],
                       seed_nreval=snr[:n_seeds])
        return out

    def retina_grid_search(self, meas_dim, plane_z, event_offsets, x, y, plane, grid: dict,
                           capacity=None, want_grid=False):
        """Grid-search Artificial Retina over the batch.  grid: n, lo, hi, sigma,
        R0.  Returns dict(tracks (structured numpy array or uint8 tensor view),
        track_offsets, R_grid ([E, n0, n1] or None))."""
        g, zkeep = self._geometry(meas_dim, plane_z)
        hits, keep, mem = self._hits(meas_dim, event_offsets, x, y, plane)
        E = hits.n_events
        n0, n1 = int(grid["n"][0]), int(grid["n"][1])
        G = Grid((ctypes.c_int32 * 2)(n0, n1), (ctypes.c_float * 2)(*grid["lo"]),
                 (ctypes.c_float * 2)(*grid["hi"]), float(grid["sigma"]), float(grid["R0"]))
        cap = E * ((n0 * n1 + 1) // 2) if capacity is None else int(capacity)
        if mem == MEM_HOST:
            tracks = np.zeros(max(cap, 1), TRACK_DTYPE)
            toff = np.zeros(E + 1, np.int64)
            Rg = np.zeros((E, n0, n1), np.float32) if want_grid else None
        else:
            import torch
            dev = x.device
            self.set_stream(torch.cuda.current_stream(dev).cuda_stream)
            tracks = torch.empty(max(cap, 1) * 48, dtype=torch.uint8, device=dev)  # records [0, offsets[-1]) written
            toff = torch.zeros(E + 1, dtype=torch.int64, device=dev)
            Rg = torch.zeros((E, n0, n1), dtype=torch.float32, device=dev) if want_grid else None
        rc = self.lib.retina_grid_search(self.h, ctypes.byref(g), ctypes.byref(hits), ctypes.byref(G),
                                         _ptr(Rg), _ptr(tracks), cap, _ptr(toff))
        if rc == ERR_CAPACITY:
            need = int(toff[-1]) if mem == MEM_HOST else int(toff[-1].item())
            err = RetinaError(rc, self.lib.retina_last_error(self.h).decode())
            err.required = need
            raise err
        self._check(rc)
        out = dict(track_offsets=toff, R_grid=Rg)
        if mem == MEM_HOST:
            out["tracks"] = tracks[:int(toff[-1])]
        else:
            out["tracks_bytes"] = tracks
        return out

    # ------------------------------------------------ learned seed proposer
    def retina_model_create(self, init_key: int) -> Model:
        h = ctypes.c_void_p()
        self._check(self.lib.retina_model_create(self.h, int(init_key), ctypes.byref(h)))
        return Model(self, h)

    def retina_model_load(self, path: str) -> Model:
        h = ctypes.c_void_p()
        self._check(self.lib.retina_model_load(self.h, path.encode(), ctypes.byref(h)))
        return Model(self, h)

    def _model_io(self, plane_z, event_offsets, x, y, plane):
        g, zkeep = self._geometry(2, plane_z)
        hits, keep, mem = self._hits(2, event_offsets, x, y, plane)
        if mem == MEM_DEVICE:
            import torch
            self.set_stream(torch.cuda.current_stream(x.device).cuda_stream)
        return g, hits, (zkeep, keep), mem

    def retina_train_step(self, model: Model, plane_z, event_offsets, x, y, plane, targets,
                          target_offsets, lr: float, pos_weight: float, want_grad=False):
        """One Adam step (lr > 0) or a gradient evaluation (lr = 0).
        Returns (loss, grad or None); grad is host FP32 in the logical layout."""
        g, hits, keep, mem = self._model_io(plane_z, event_offsets, x, y, plane)
        if mem == MEM_HOST:
            tg = _host(targets, np.float64).reshape(-1, 2)
            to = _host(target_offsets, np.int64)
        else:
            import torch
            tg = _dev(targets, torch.float64)
            to = _dev(target_offsets, torch.int64)
        loss = ctypes.c_float()
        grad = np.zeros(MODEL_PARAMS, np.float32) if want_grad else None
        self._check(self.lib.retina_train_step(self.h, model.h, ctypes.byref(g), ctypes.byref(hits),
                                               _ptr(tg), _ptr(to), float(lr), float(pos_weight),
                                               ctypes.byref(loss), _ptr(grad)))
        return loss.value, grad

    def retina_model_forward(self, model: Model, plane_z, event_offsets, x, y, plane):
        """Binned images (uint16 BF16 bits, [E, 128, 128, 2]) and logits ([E, 128, 128])."""
        g, hits, keep, mem = self._model_io(plane_z, event_offsets, x, y, plane)
        E = hits.n_events
        if mem == MEM_HOST:
            img = np.zeros((E, IMG, IMG, 2), np.uint16)
            logits = np.zeros((E, IMG, IMG), np.float32)
        else:
            import torch
            img = torch.zeros((E, IMG, IMG, 2), dtype=torch.int16, device=x.device)
            logits = torch.zeros((E, IMG, IMG), dtype=torch.float32, device=x.device)
        self._check(self.lib.retina_model_forward(self.h, model.h, ctypes.byref(g), ctypes.byref(hits),
                                                  _ptr(img), _ptr(logits)))
        return img, logits

    def retina_propose_seeds(self, model: Model, plane_z, event_offsets, x, y, plane, k_max: int,
                             tau: float, conf_min: float, params: dict, capacity=None, nms: bool = False):
        """Seeds from the network (lattice fallback per event).  Returns dict(seeds
        [n, 4], seed_offsets, confidence, fallback)."""
        g, hits, keep, mem = self._model_io(plane_z, event_offsets, x, y, plane)
        E = hits.n_events
        P, pkeep, _ = self._params(params, None, None, mem, 4, E)
        lat = params["lattice_n"][0] * params["lattice_n"][1]
        cap = E * max(int(k_max), lat) if capacity is None else int(capacity)
        if mem == MEM_HOST:
            seeds = np.zeros((max(cap, 1), 4))
            so = np.zeros(E + 1, np.int64)
            conf = np.zeros(max(E, 1), np.float32)
            fb = np.zeros(max(E, 1), np.int32)
        else:
            import torch
            dev = x.device
            seeds = torch.zeros((max(cap, 1), 4), dtype=torch.float64, device=dev)
            so = torch.zeros(E + 1, dtype=torch.int64, device=dev)
            conf = torch.zeros(max(E, 1), dtype=torch.float32, device=dev)
            fb = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        pr = Proposal(int(k_max), float(tau), float(conf_min), int(bool(nms)))
        rc = self.lib.retina_propose_seeds(self.h, ctypes.byref(g), ctypes.byref(hits), model.h, ctypes.byref(pr),
                                           ctypes.byref(P), _ptr(seeds), cap, _ptr(so), _ptr(conf), _ptr(fb))
        if rc == ERR_CAPACITY:
            err = RetinaError(rc, self.lib.retina_last_error(self.h).decode())
            err.required = int(so[-1]) if mem == MEM_HOST else int(so[-1].item())
            raise err
        self._check(rc)
        n = int(so[-1]) if mem == MEM_HOST else int(so[-1].item())
        return dict(seeds=seeds[:n], seed_offsets=so, confidence=conf[:E], fallback=fb[:E])

    def retina_find_tracks_learned(self, model: Model, plane_z, event_offsets, x, y, plane, params: dict,
                                   k_max: int, tau: float, conf_min: float, capacity=None, nms: bool = False):
        """Algorithm 1 on learned seeds.  Same result layout as retina_find_tracks."""
        g, hits, keep, mem = self._model_io(plane_z, event_offsets, x, y, plane)
        E = hits.n_events
        P, pkeep, _ = self._params(params, None, None, mem, 4, E)
        lat = params["lattice_n"][0] * params["lattice_n"][1]
        cap = E * max(int(k_max), lat) if capacity is None else int(capacity)
        if mem == MEM_HOST:
            tracks = np.zeros(max(cap, 1), TRACK_DTYPE)
            toff = np.zeros(E + 1, np.int64)
            evf = np.zeros(max(E, 1), np.int32)
        else:
            import torch
            dev = x.device
            tracks = torch.empty(max(cap, 1) * 48, dtype=torch.uint8, device=dev)  # records [0, offsets[-1]) written
            toff = torch.zeros(E + 1, dtype=torch.int64, device=dev)
            evf = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        pr = Proposal(int(k_max), float(tau), float(conf_min), int(bool(nms)))
        rc = self.lib.retina_find_tracks_learned(self.h, ctypes.byref(g), ctypes.byref(hits), ctypes.byref(P),
                                                 model.h, ctypes.byref(pr), _ptr(tracks), cap, _ptr(toff),
                                                 _ptr(evf))
        if rc == ERR_CAPACITY:
            err = RetinaError(rc, self.lib.retina_last_error(self.h).decode())
            err.required = int(toff[-1]) if mem == MEM_HOST else int(toff[-1].item())
            raise err
        self._check(rc)
        out = dict(track_offsets=toff, event_flags=evf[:E])
        if mem == MEM_HOST:
            out["tracks"] = tracks[:int(toff[-1])]
        else:
            out["tracks_bytes"] = tracks
        return out


def tracks_from_device(res) -> np.ndarray:
    """Copy a device-memory find_tracks result's tracks to a structured array."""
    raw = res["tracks_bytes"].cpu().numpy()
    n = int(res["track_offsets"][-1].item())
    return raw[: n * 48].view(TRACK_DTYPE)


class Model:
    """Handle of a retina_model (learned seed proposer) on a context's device."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.h = handle

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.retina_model_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step(self) -> int:
        return int(self.ctx.lib.retina_model_step(self.h))

    def retina_model_get_params(self) -> np.ndarray:
        out = np.zeros(MODEL_PARAMS, np.float32)
        self.ctx._check(self.ctx.lib.retina_model_get_params(self.h, _ptr(out)))
        return out

    def retina_model_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MODEL_PARAMS,):
            raise ValueError("expected %d parameters" % MODEL_PARAMS)
        self.ctx._check(self.ctx.lib.retina_model_set_params(self.h, _ptr(p)))

    def retina_model_save(self, path: str):
        self.ctx._check(self.ctx.lib.retina_model_save(self.h, path.encode()))
