"""The simplified VELO of Section 3 (generator and prior draws) and the
origin-constrained ascent on it: pins of the oracle's slope-block polish by
the weighted least-squares fixed point through the origin."""
import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events


@pytest.fixture(scope="module")
def cfg():
    return events.load_config("c8")


def test_svelo_generator(cfg):
    zp = events.plane_z(cfg)
    assert zp.shape == (20,) and zp[0] == 35.0 and zp[-1] == 700.0
    sv = cfg["svelo"]
    n_noise, hits_per_track = [], []
    for i in range(20):
        ev = events.make_event(cfg, i, zp)
        assert ev.truth.shape == (200, 4) and np.all(ev.truth[:, :2] == 0)
        assert np.all(ev.truth_nhits >= sv["n_min"])
        tt = np.hypot(ev.truth[:, 2], ev.truth[:, 3])
        eta = -np.log(np.tan(np.arctan(tt) / 2))
        assert eta.min() >= 1.0 and eta.max() <= 6.0
        r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
        assert r.min() >= sv["r_inner"] - 0.1 and r.max() <= sv["r_outer"] + 0.1   # disks (+ smearing)
        for k in range(0, 200, 37):   # track hits lie on their line within the smearing
            m = ev.label == k
            z = zp[ev.plane[m]].astype(np.float64)
            res = np.concatenate([ev.x[m] - ev.truth[k, 2] * z, ev.y[m] - ev.truth[k, 3] * z])
            assert np.abs(res).max() < 6 * sv["smear_sd"]
            assert m.sum() == ev.truth_nhits[k]
        n_noise.append(int(np.sum(ev.label == -1)))
        hits_per_track.append(ev.truth_nhits.mean())
    # noise: Poisson(250) plus the hits of particles with fewer than 2 hits
    assert 250 < np.mean(n_noise) < 400
    assert 3.5 < np.mean(hits_per_track) < 7


def test_prior_seeds(cfg):
    s, off = events.prior_seeds(cfg, 5000, [3, 4])
    assert s.shape == (10000, 4) and list(off) == [0, 5000, 10000] and np.all(s[:, :2] == 0)
    tt = np.hypot(s[:, 2], s[:, 3])
    eta = -np.log(np.tan(np.arctan(tt) / 2))
    assert 1.0 <= eta.min() and eta.max() <= 6.0
    assert abs(np.mean(eta) - 3.5) < 0.05                      # uniform in eta
    s2, _ = events.prior_seeds(cfg, 5000, [4])
    np.testing.assert_array_equal(s2, s[5000:])               # keyed by event index


def test_origin_constrained_maximum_is_weighted_lsq_through_origin(cfg):
    """With the offsets held through the steps and the polish, a converged
    maximum satisfies the slope block's stationarity: (tx, ty) is the weighted
    least-squares line through the origin with weights e_k at the solution,
    tx = sum e x z / sum e z^2 (likewise ty), and x0 = y0 = 0 exactly."""
    zp = events.plane_z(cfg)
    ev = events.make_event(cfg, 7, zp)
    b = events.batch_from_events(2, zp, [ev])
    P = dict(cfg["params"])
    assert P["n_slope_steps"] >= len(P["sigma"]) + P["n_final_steps"] + P["n_polish"]
    seeds = ev.truth[:40].copy()
    seeds[:, 2:] += np.random.default_rng(1).normal(0, 2e-3, (40, 2))
    res = oracle.find_tracks(b, P, seeds=seeds, seed_offsets=np.array([0, 40]))
    th, fl = res["seed_theta"], res["seed_flags"]
    assert np.all(th[:, :2] == 0.0)
    z = zp[ev.plane].astype(np.float64)
    x, y = ev.x.astype(np.float64), ev.y.astype(np.float64)
    s2 = P["sigma_final"] ** 2
    n_conv = 0
    for t, f in zip(th, fl):
        if not f & 1:
            continue
        n_conv += 1
        e = np.exp(-((x - t[2] * z) ** 2 + (y - t[3] * z) ** 2) / s2)
        wz2 = np.sum(e * z * z)
        assert t[2] == pytest.approx(np.sum(e * x * z) / wz2, rel=1e-9, abs=1e-12)
        assert t[3] == pytest.approx(np.sum(e * y * z) / wz2, rel=1e-9, abs=1e-12)
    assert n_conv >= 30


def test_full_four_parameter_polish_moves_offsets(cfg):
    """Control for the pin above: the same seeds with a four-parameter polish
    (n_slope_steps inside the steps) end with non-zero offsets."""
    zp = events.plane_z(cfg)
    ev = events.make_event(cfg, 7, zp)
    b = events.batch_from_events(2, zp, [ev])
    P = dict(cfg["params"], n_slope_steps=4)
    res = oracle.find_tracks(b, P, seeds=ev.truth[:10], seed_offsets=np.array([0, 10]))
    assert np.any(res["seed_theta"][:, :2] != 0.0)
