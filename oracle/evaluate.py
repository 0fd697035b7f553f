"""Track-finding evaluation against generator truth (plain definitions).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

A found track matches a true track when their largest in-plane separation
over the detector's end planes is within ``tol``; matching is greedy, nearest
pair first, one found track per true track.  Section 3 defines a track as
reconstructed when an estimate lies within eps = 1e-3 of the true parameters;
on slopes that criterion is reported too (``eff_eps``).
"""
from __future__ import annotations

import numpy as np


def _dist(meas_dim, a, b, z_first, z_last):
    """[na, nb] largest end-plane separation between two sets of lines."""
    a = np.atleast_2d(a)[:, None, :]
    b = np.atleast_2d(b)[None, :, :]
    d = np.zeros((a.shape[0], b.shape[1]))
    for z in (z_first, z_last):
        if meas_dim == 2:
            dx = np.abs((a[..., 0] - b[..., 0]) + (a[..., 2] - b[..., 2]) * z)
            dy = np.abs((a[..., 1] - b[..., 1]) + (a[..., 3] - b[..., 3]) * z)
            d = np.maximum(d, np.maximum(dx, dy))
        else:
            d = np.maximum(d, np.abs((a[..., 0] - b[..., 0]) + (a[..., 1] - b[..., 1]) * z))
    return d


def match_tracks(meas_dim, found, truth, tol, z_first, z_last):
    """Greedy nearest-first matching.  Returns (found->true index or -1,
    true->found index or -1, pairwise distance matrix)."""
    found = np.asarray(found, np.float64).reshape(-1, 2 * meas_dim)
    truth = np.asarray(truth, np.float64).reshape(-1, 2 * meas_dim)
    f2t = np.full(found.shape[0], -1, np.int64)
    t2f = np.full(truth.shape[0], -1, np.int64)
    if found.shape[0] == 0 or truth.shape[0] == 0:
        return f2t, t2f, np.zeros((found.shape[0], truth.shape[0]))
    d = _dist(meas_dim, found, truth, z_first, z_last)
    order = np.argsort(d, axis=None, kind="stable")
    for flat in order:
        i, j = divmod(int(flat), truth.shape[0])
        if d[i, j] > tol:
            break
        if f2t[i] < 0 and t2f[j] < 0:
            f2t[i] = j
            t2f[j] = i
    return f2t, t2f, d


def efficiency(meas_dim, found, truth, truth_nhits, tol, z_first, z_last, n_min=2, eps=1e-3):
    """Efficiency / fake / clone counts for one event (see module docstring)."""
    found = np.asarray(found, np.float64).reshape(-1, 2 * meas_dim)
    truth = np.asarray(truth, np.float64).reshape(-1, 2 * meas_dim)
    rec = np.asarray(truth_nhits) >= n_min
    f2t, t2f, d = match_tracks(meas_dim, found, truth, tol, z_first, z_last)
    n_found = found.shape[0]
    matched_rec = int(np.sum((t2f >= 0) & rec))
    near_any = (d <= tol).any(axis=1) if d.size else np.zeros(n_found, bool)
    clones = int(np.sum((f2t < 0) & near_any))
    fakes = int(np.sum(~near_any))
    # paper's criterion on slopes: some found track within eps in both slopes
    sl = slice(2, 4) if meas_dim == 2 else slice(1, 2)
    if n_found and truth.shape[0]:
        ds = np.max(np.abs(found[:, None, sl] - truth[None, :, sl]), axis=2)
        eps_ok = (ds <= eps).any(axis=0)
    else:
        eps_ok = np.zeros(truth.shape[0], bool)
    return dict(n_true_rec=int(rec.sum()), n_matched=matched_rec, n_found=n_found,
                n_fake=fakes, n_clone=clones, n_eps=int(np.sum(eps_ok & rec)))


def summarize(stats: list) -> dict:
    """Sum per-event counts into rates."""
    tot = {k: sum(s[k] for s in stats) for k in stats[0]} if stats else {}
    if not tot:
        return {}
    return dict(efficiency=tot["n_matched"] / max(tot["n_true_rec"], 1),
                fake_rate=tot["n_fake"] / max(tot["n_found"], 1),
                clone_rate=tot["n_clone"] / max(tot["n_found"], 1),
                eff_eps=tot["n_eps"] / max(tot["n_true_rec"], 1), **tot)
