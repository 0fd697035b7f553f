"""Track-finding quality against generator truth, for the benchmark report.

A found line and a true line match when their in-plane separation at both end
planes of the detector is within `tol` in every measured coordinate (the
separation is linear in z, so the two end planes bound it everywhere inside).
Each true track takes at most one found track, nearest pairs first.

  efficiency  matched reconstructible true tracks / reconstructible true tracks
              (reconstructible: at least 2 hits, as in Section 3)
  fake rate   found tracks within tol of no true track / found tracks
  clone rate  further found tracks within tol of an already matched true track
              / found tracks
  eff_eps     Section 3's criterion: some found track within 1e-3 of the true
              slopes (max over the slope components)
  fake_rate_eps  found tracks whose slopes are within 1e-3 of no true track
              / found tracks (the same criterion, for estimates that carry
              slopes only, such as the grid search's)
  eff_angle   for tracks from the origin (the simplified VELO): some found
              track whose direction (tx, ty, 1) lies within 1e-3 rad of the
              true direction; fake_rate_angle likewise
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def _endpoints(theta: np.ndarray, meas_dim: int, z0: float, z1: float) -> np.ndarray:
    """Lines -> their coordinates at the two end planes, [n, 2*meas_dim]."""
    t = np.asarray(theta, np.float64).reshape(-1, 2 * meas_dim)
    off, slope = t[:, :meas_dim], t[:, meas_dim:]
    return np.concatenate([off + slope * z0, off + slope * z1], axis=1)


def _close_pairs(a, b, r, p):
    """Pairs (i, j) with |a[i] - b[j]| <= r in the p-norm (KD-trees), with the
    distances."""
    if a.shape[0] == 0 or b.shape[0] == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    m = cKDTree(a).sparse_distance_matrix(cKDTree(b), r, p=p, output_type="ndarray")
    return m["i"].astype(np.int64), m["j"].astype(np.int64), m["v"]


def _unit_directions(slopes):
    u = np.concatenate([slopes, np.ones((slopes.shape[0], 1))], axis=1)
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def event_quality(meas_dim, found, truth, truth_nhits, tol, z0, z1, eps=1e-3):
    pf = _endpoints(found, meas_dim, z0, z1)
    pt = _endpoints(truth, meas_dim, z0, z1)
    nf, nt = pf.shape[0], pt.shape[0]
    rec = np.asarray(truth_nhits) >= 2
    out = dict(n_true_rec=int(rec.sum()), n_found=nf, n_matched=0, n_fake=nf, n_clone=0, n_eps=0, n_fake_eps=nf,
               n_ang=0, n_fake_ang=nf)
    if nf == 0 or nt == 0:
        return out
    # end-plane separation (Chebyshev) within tol; greedy, nearest pairs first,
    # ties in (found, true) index order
    fi, ti, cheb = _close_pairs(pf, pt, tol, np.inf)
    used_f = np.zeros(nf, bool)
    used_t = np.zeros(nt, bool)
    for k in np.lexsort((ti, fi, cheb)):
        f, t = fi[k], ti[k]
        if not used_f[f] and not used_t[t]:
            used_f[f] = used_t[t] = True
    near_any = np.zeros(nf, bool)
    near_any[fi] = True
    slopes_f = np.asarray(found, np.float64).reshape(nf, -1)[:, meas_dim:]
    slopes_t = np.asarray(truth, np.float64).reshape(nt, -1)[:, meas_dim:]
    ef, et, _ = _close_pairs(slopes_f, slopes_t, eps, np.inf)
    eps_t = np.zeros(nt, bool)
    eps_t[et] = True
    eps_f = np.zeros(nf, bool)
    eps_f[ef] = True
    if meas_dim == 2:
        # angle between directions <= eps  <=>  chord between unit vectors <= 2 sin(eps / 2)
        af, at, _ = _close_pairs(_unit_directions(slopes_f), _unit_directions(slopes_t), 2.0 * np.sin(eps / 2.0), 2)
        ang_t = np.zeros(nt, bool)
        ang_t[at] = True
        ang_f = np.zeros(nf, bool)
        ang_f[af] = True
    else:
        ang_t, ang_f = eps_t, eps_f
    out.update(n_matched=int((used_t & rec).sum()), n_fake=int((~near_any).sum()),
               n_clone=int((near_any & ~used_f).sum()), n_eps=int((eps_t & rec).sum()),
               n_fake_eps=int((~eps_f).sum()), n_ang=int((ang_t & rec).sum()), n_fake_ang=int((~ang_f).sum()))
    return out


def batch_quality(meas_dim, tracks_theta, track_offsets, truth_list, truth_nhits_list, tol, z0, z1):
    tot = dict(n_true_rec=0, n_found=0, n_matched=0, n_fake=0, n_clone=0, n_eps=0, n_fake_eps=0, n_ang=0,
               n_fake_ang=0)
    off = np.asarray(track_offsets)
    for e in range(len(truth_list)):
        q = event_quality(meas_dim, tracks_theta[off[e]:off[e + 1]], truth_list[e], truth_nhits_list[e],
                          tol, z0, z1)
        for k in tot:
            tot[k] += q[k]
    rec = max(tot["n_true_rec"], 1)
    nf = max(tot["n_found"], 1)
    return dict(efficiency=tot["n_matched"] / rec, fake_rate=tot["n_fake"] / nf,
                clone_rate=tot["n_clone"] / nf, eff_eps=tot["n_eps"] / rec, fake_rate_eps=tot["n_fake_eps"] / nf,
                eff_angle=tot["n_ang"] / rec, fake_rate_angle=tot["n_fake_ang"] / nf, **tot)
