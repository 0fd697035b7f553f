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


def _endpoints(theta: np.ndarray, meas_dim: int, z0: float, z1: float) -> np.ndarray:
    """Lines -> their coordinates at the two end planes, [n, 2*meas_dim]."""
    t = np.asarray(theta, np.float64).reshape(-1, 2 * meas_dim)
    off, slope = t[:, :meas_dim], t[:, meas_dim:]
    return np.concatenate([off + slope * z0, off + slope * z1], axis=1)


def _direction_angle(sf, st):
    """Angle between the directions (tx, ty, 1) of every found / true pair."""
    u = np.concatenate([sf, np.ones((sf.shape[0], 1))], axis=1)
    v = np.concatenate([st, np.ones((st.shape[0], 1))], axis=1)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    chord = np.linalg.norm(u[:, None, :] - v[None, :, :], axis=2)
    return 2.0 * np.arcsin(np.minimum(chord / 2.0, 1.0))


def event_quality(meas_dim, found, truth, truth_nhits, tol, z0, z1, eps=1e-3):
    pf = _endpoints(found, meas_dim, z0, z1)
    pt = _endpoints(truth, meas_dim, z0, z1)
    nf, nt = pf.shape[0], pt.shape[0]
    rec = np.asarray(truth_nhits) >= 2
    out = dict(n_true_rec=int(rec.sum()), n_found=nf, n_matched=0, n_fake=nf, n_clone=0, n_eps=0, n_fake_eps=nf,
               n_ang=0, n_fake_ang=nf)
    if nf == 0 or nt == 0:
        return out
    cheb = np.abs(pf[:, None, :] - pt[None, :, :]).max(axis=2)  # Chebyshev separation
    close = cheb <= tol
    fi, ti = np.nonzero(close)
    order = np.argsort(cheb[fi, ti], kind="stable")
    used_f = np.zeros(nf, bool)
    used_t = np.zeros(nt, bool)
    for k in order:
        f, t = fi[k], ti[k]
        if not used_f[f] and not used_t[t]:
            used_f[f] = used_t[t] = True
    near_any = close.any(axis=1)
    slopes_f = np.asarray(found, np.float64).reshape(nf, -1)[:, meas_dim:]
    slopes_t = np.asarray(truth, np.float64).reshape(nt, -1)[:, meas_dim:]
    eps_close = np.abs(slopes_f[:, None, :] - slopes_t[None, :, :]).max(axis=2) <= eps
    eps_ok = eps_close.any(axis=0)
    ang_close = _direction_angle(slopes_f, slopes_t) <= eps if meas_dim == 2 else eps_close
    out.update(n_matched=int((used_t & rec).sum()), n_fake=int((~near_any).sum()),
               n_clone=int((near_any & ~used_f).sum()), n_eps=int((eps_ok & rec).sum()),
               n_fake_eps=int((~eps_close.any(axis=1)).sum()), n_ang=int((ang_close.any(axis=0) & rec).sum()),
               n_fake_ang=int((~ang_close.any(axis=1)).sum()))
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
