"""Seeded synthetic event generator (the input side only).

This module draws detector hits and their truth; it holds none of the track
finder's arithmetic (no response, no seeds, no fitting), so both the HIP path
and the FP64 CPU oracle may consume what it produces.

The detector follows the paper's simplified VELO model (Section 3): planes
perpendicular to the beam axis z, straight tracks, Gaussian smearing of the
in-plane coordinates and uniformly distributed noise hits.  The concrete
workloads (plane positions, track counts, slope ranges, inefficiency, noise
fractions) are the JSON files in ``configs/``; each field there is a stated
choice where the paper leaves the workload open.

Random streams: every event uses its own ``numpy.random.Philox`` keyed by
``(config key, event index)``, so any event can be regenerated alone and in any
order.  Coordinates are drawn in FP64 and rounded once to FP32, which is the
hit precision both sides consume.

Measurement dimension:
  * ``meas_dim == 2``: a hit is (plane, x, y); a track is (x0, y0, tx, ty) with
    x(z) = x0 + tx*z and y(z) = y0 + ty*z.
  * ``meas_dim == 1``: the 2D toy of Section 2 / Fig. 1.  Planes sit at
    positions z (the paper's x); a hit carries one measured coordinate u (the
    paper's y) stored in ``x``; a track is (x0, tx) = (beta, alpha) with
    u(z) = x0 + tx*z.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Optional

import numpy as np

_CFG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def load_config(name: str) -> dict:
    """Load a workload description (``c1`` .. ``c5``) from ``configs/``."""
    path = name if name.endswith(".json") else os.path.join(_CFG_DIR, name + ".json")
    with open(path) as f:
        return json.load(f)


def plane_z(cfg: dict) -> np.ndarray:
    """Plane positions along z as FP32 (equally spaced for the VELO-like configs)."""
    pl = cfg["planes"]
    if pl["kind"] == "list":
        z = np.asarray(pl["z"], dtype=np.float64)
    elif pl["kind"] == "uniform":
        n = int(pl["n"])
        z = pl["z_first"] + (pl["z_last"] - pl["z_first"]) * np.arange(n, dtype=np.float64) / (n - 1)
    else:
        raise ValueError("unknown plane kind %r" % pl["kind"])
    return z.astype(np.float32)


@dataclasses.dataclass
class Event:
    x: np.ndarray          # float32 [n_hits]
    y: Optional[np.ndarray]  # float32 [n_hits] or None for meas_dim 1
    plane: np.ndarray      # int32 [n_hits]
    label: np.ndarray      # int32 [n_hits], index of the generating track, -1 for noise
    truth: np.ndarray      # float64 [n_tracks, 2*meas_dim]: (x0, tx) or (x0, y0, tx, ty)
    truth_nhits: np.ndarray  # int32 [n_tracks]

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class Batch:
    meas_dim: int
    plane_z: np.ndarray          # float32 [n_planes]
    event_offsets: np.ndarray    # int64 [n_events+1]
    x: np.ndarray                # float32 [total_hits]
    y: Optional[np.ndarray]      # float32 [total_hits] or None
    plane: np.ndarray            # int32 [total_hits]
    label: np.ndarray            # int32 [total_hits]
    truth: list                  # per event float64 arrays
    truth_nhits: list            # per event int32 arrays
    index: Optional[list] = None  # event indices in the config's stream (scan batches)

    @property
    def n_events(self) -> int:
        return int(self.event_offsets.shape[0] - 1)

    def event(self, e: int) -> Event:
        a, b = int(self.event_offsets[e]), int(self.event_offsets[e + 1])
        return Event(self.x[a:b], None if self.y is None else self.y[a:b], self.plane[a:b],
                     self.label[a:b], self.truth[e], self.truth_nhits[e])


def _rng(cfg: dict, idx: int) -> np.random.Generator:
    key = np.array([int(cfg["key"]), int(idx)], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def _draw_param(rng, spec, n):
    if spec["kind"] == "uniform":
        return rng.uniform(spec["lo"], spec["hi"], n)
    if spec["kind"] == "normal":
        return rng.normal(0.0, spec["sd"], n)
    raise ValueError("unknown distribution %r" % spec["kind"])


def _make_svelo_event(cfg: dict, idx: int, zp: np.ndarray) -> Event:
    """The simplified VELO of Section 3: disk layers perpendicular to z, tracks
    from the origin with pseudo-rapidity eta ~ U[eta_lo, eta_hi] (polar angle
    theta = 2 atan(exp(-eta))) and azimuth phi ~ U[0, 2 pi), direction
    (sin theta cos phi, sin theta sin phi, cos theta); a layer records the
    crossing with probability p_hit when it lies on the disk (r_inner <= r <=
    r_outer), smeared by N(0, sd) in x and y.  Particles are drawn until
    `count` of them leave at least n_min hits; the hits of the others are kept
    as noise (label -1), as are Poisson(noise_mean) hits uniform in area on a
    uniformly chosen layer.  Truth: (x0, y0, tx, ty) = (0, 0, tan theta cos phi,
    tan theta sin phi) of the reconstructible tracks."""
    rng = _rng(cfg, idx)
    sv = cfg["svelo"]
    z64 = zp.astype(np.float64)
    n_planes = zp.shape[0]
    target = int(cfg["tracks"]["count"]["n"])
    r_in, r_out = float(sv["r_inner"]), float(sv["r_outer"])
    sd, p_hit, n_min = float(sv["smear_sd"]), float(sv["p_hit"]), int(sv["n_min"])
    truth, nh, hx, hy, hp, hl = [], [], [], [], [], []
    n_rec = 0
    while n_rec < target:
        m = 2 * (target - n_rec) + 16   # one chunk of particles, consumed in order
        eta = rng.uniform(sv["eta"][0], sv["eta"][1], m)
        phi = rng.uniform(0.0, 2.0 * np.pi, m)
        ran = rng.random((m, n_planes))
        ex = rng.normal(0.0, sd, (m, n_planes))
        ey = rng.normal(0.0, sd, (m, n_planes))
        tt = np.tan(2.0 * np.arctan(np.exp(-eta)))
        tx, ty = tt * np.cos(phi), tt * np.sin(phi)
        r = tt[:, None] * z64[None, :]
        hit = (r >= r_in) & (r <= r_out) & (ran < p_hit)
        for k in range(m):
            if n_rec == target:
                break
            lay = np.nonzero(hit[k])[0]
            rec = lay.size >= n_min
            hx.append(tx[k] * z64[lay] + ex[k, lay])
            hy.append(ty[k] * z64[lay] + ey[k, lay])
            hp.append(lay.astype(np.int32))
            hl.append(np.full(lay.size, n_rec if rec else -1, np.int32))
            if rec:
                truth.append((0.0, 0.0, tx[k], ty[k]))
                nh.append(lay.size)
                n_rec += 1
    n_noise = int(rng.poisson(float(sv["noise_mean"])))
    nr = np.sqrt(rng.uniform(r_in * r_in, r_out * r_out, n_noise))
    na = rng.uniform(0.0, 2.0 * np.pi, n_noise)
    hx.append(nr * np.cos(na))
    hy.append(nr * np.sin(na))
    hp.append(rng.integers(0, n_planes, n_noise).astype(np.int32))
    hl.append(np.full(n_noise, -1, np.int32))
    x, y = np.concatenate(hx), np.concatenate(hy)
    plane, label = np.concatenate(hp).astype(np.int32), np.concatenate(hl).astype(np.int32)
    perm = rng.permutation(x.shape[0])
    return Event(x=x[perm].astype(np.float32), y=y[perm].astype(np.float32), plane=plane[perm],
                 label=label[perm], truth=np.array(truth, np.float64).reshape(-1, 4),
                 truth_nhits=np.array(nh, np.int32))


def prior_seeds(cfg: dict, n: int, events_idx) -> tuple:
    """Algorithm 1's first step for the simplified VELO: n initial guesses per
    event drawn from the track prior (eta ~ U[eta_lo, eta_hi], phi ~ U[0, 2 pi)),
    as lines from the origin (0, 0, tan theta cos phi, tan theta sin phi).  The
    draws of event index i come from their own Philox stream keyed by
    (seed key, i); slopes are rounded to FP32, the precision the GPU path starts
    from.  Returns (seeds [len(events_idx) * n, 4] float64, offsets)."""
    sv = cfg["svelo"]
    out = np.zeros((len(events_idx) * n, 4))
    for k, i in enumerate(events_idx):
        key = np.array([int(cfg["seed_key"]), int(i)], dtype=np.uint64)
        rng = np.random.Generator(np.random.Philox(key=key))
        eta = rng.uniform(sv["eta"][0], sv["eta"][1], n)
        phi = rng.uniform(0.0, 2.0 * np.pi, n)
        tt = np.tan(2.0 * np.arctan(np.exp(-eta)))
        out[k * n:(k + 1) * n, 2] = (tt * np.cos(phi)).astype(np.float32)
        out[k * n:(k + 1) * n, 3] = (tt * np.sin(phi)).astype(np.float32)
    return out, np.arange(len(events_idx) + 1, dtype=np.int64) * n


def make_event(cfg: dict, idx: int, zp: Optional[np.ndarray] = None) -> Event:
    """Generate event ``idx`` of workload ``cfg`` (deterministic in (key, idx))."""
    if cfg.get("kind") == "svelo":
        return _make_svelo_event(cfg, idx, plane_z(cfg) if zp is None else zp)
    rng = _rng(cfg, idx)
    D = int(cfg["meas_dim"])
    if zp is None:
        zp = plane_z(cfg)
    z64 = zp.astype(np.float64)
    n_planes = zp.shape[0]
    tr = cfg["tracks"]

    cnt = tr["count"]
    if cnt["kind"] == "fixed":
        n_tracks = int(cnt["n"])
    elif cnt["kind"] == "poisson":
        n_tracks = int(np.clip(rng.poisson(cnt["mean"]), cnt["lo"], cnt["hi"]))
    else:
        raise ValueError("unknown count kind %r" % cnt["kind"])

    if D == 2:
        x0 = _draw_param(rng, tr["x0"], n_tracks)
        y0 = _draw_param(rng, tr["x0"], n_tracks)
        tx = _draw_param(rng, tr["tx"], n_tracks)
        ty = _draw_param(rng, tr["tx"], n_tracks)
        truth = np.stack([x0, y0, tx, ty], axis=1)
    else:
        x0 = _draw_param(rng, tr["x0"], n_tracks)
        tx = _draw_param(rng, tr["tx"], n_tracks)
        truth = np.stack([x0, tx], axis=1)

    # one candidate hit per (track, plane); inefficiency drops each independently
    sd = float(tr["smear_sd"])
    keep = rng.random((n_tracks, n_planes)) >= float(tr["inefficiency"])
    hx = x0[:, None] + tx[:, None] * z64[None, :] + rng.normal(0.0, sd, (n_tracks, n_planes))
    if D == 2:
        hy = y0[:, None] + ty[:, None] * z64[None, :] + rng.normal(0.0, sd, (n_tracks, n_planes))
    tid = np.broadcast_to(np.arange(n_tracks, dtype=np.int32)[:, None], (n_tracks, n_planes))
    pid = np.broadcast_to(np.arange(n_planes, dtype=np.int32)[None, :], (n_tracks, n_planes))
    tx_hits = hx[keep]
    ty_hits = hy[keep] if D == 2 else None
    t_lab = tid[keep]
    t_pl = pid[keep]
    truth_nhits = keep.sum(axis=1).astype(np.int32)
    n_true = int(t_lab.shape[0])

    nz = cfg["noise"]
    if nz["kind"] == "count":
        n_noise = int(nz["n"])
    elif nz["kind"] == "fraction":
        n_noise = int(round(float(nz["f"]) * n_true))
    elif nz["kind"] == "fraction_uniform":
        f = rng.uniform(nz["f_lo"], nz["f_hi"])
        n_noise = int(round(f * n_true))
    else:
        raise ValueError("unknown noise kind %r" % nz["kind"])
    n_pl = rng.integers(0, n_planes, n_noise).astype(np.int32)
    n_x = rng.uniform(nz["lo"], nz["hi"], n_noise)
    n_y = rng.uniform(nz["lo"], nz["hi"], n_noise) if D == 2 else None

    x = np.concatenate([tx_hits, n_x])
    y = np.concatenate([ty_hits, n_y]) if D == 2 else None
    plane = np.concatenate([t_pl, n_pl]).astype(np.int32)
    label = np.concatenate([t_lab, np.full(n_noise, -1, np.int32)]).astype(np.int32)
    perm = rng.permutation(x.shape[0])
    return Event(
        x=x[perm].astype(np.float32),
        y=None if y is None else y[perm].astype(np.float32),
        plane=plane[perm], label=label[perm], truth=truth, truth_nhits=truth_nhits)


def make_batch(cfg: dict, n_events: Optional[int] = None, start: int = 0) -> Batch:
    """Events ``start .. start+n_events-1`` of ``cfg`` concatenated in CSR form."""
    if n_events is None:
        n_events = int(cfg["n_events"]) - start
    zp = plane_z(cfg)
    evs = [make_event(cfg, start + i, zp) for i in range(n_events)]
    return batch_from_events(int(cfg["meas_dim"]), zp, evs)


def scan_batches(cfg: dict, n_tracks=None, events_per_point: Optional[int] = None) -> list:
    """Track-count scan of a config with a ``scan`` entry: for the k-th count N,
    events k*m .. k*m+m-1 of the config's random stream, each with exactly N
    tracks (m events per point).  Returns [(N, Batch), ...]."""
    sc = cfg["scan"]
    counts = list(sc["n_tracks"])
    m = int(events_per_point or sc["events_per_point"])
    zp = plane_z(cfg)
    out = []
    for k, n in enumerate(counts):
        if n_tracks is not None and n not in n_tracks:
            continue
        c = json.loads(json.dumps(cfg))
        c["tracks"]["count"] = {"kind": "fixed", "n": int(n)}
        idx = [k * int(sc["events_per_point"]) + i for i in range(m)]
        b = batch_from_events(int(cfg["meas_dim"]), zp, [make_event(c, i, zp) for i in idx])
        b.index = idx
        out.append((int(n), b))
    return out


def batch_from_events(meas_dim: int, zp: np.ndarray, evs: list) -> Batch:
    off = np.zeros(len(evs) + 1, np.int64)
    off[1:] = np.cumsum([e.n_hits for e in evs])
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    return Batch(
        meas_dim=meas_dim, plane_z=np.asarray(zp, np.float32), event_offsets=off,
        x=cat([e.x for e in evs]).astype(np.float32),
        y=None if meas_dim == 1 else cat([e.y for e in evs]).astype(np.float32),
        plane=cat([e.plane for e in evs]).astype(np.int32),
        label=cat([e.label for e in evs]).astype(np.int32),
        truth=[e.truth for e in evs], truth_nhits=[e.truth_nhits for e in evs])


def reconstructible(ev: Event, n_min: int = 2) -> np.ndarray:
    """Mask of true tracks with at least ``n_min`` hits (Section 3: N_min = 2)."""
    return ev.truth_nhits >= n_min
