"""Pins of the oracle's step logic inside one trajectory (Algorithm 1's inner
loop with Section 3's truncated Newton and bandwidth schedule): the Armijo
acceptance rule, the halving order of the step lengths, the trial count, the
stall flag with theta left unchanged, the count of R-only evaluations, the
shortcut for short Newton steps, and the order in which the bandwidths of the
schedule are used.

Every case is a one-hit event with meas_dim 1, where the whole method reduces
to a scalar problem that can be followed by hand.  With one hit (u on the
plane at z) and a line theta = (x0, tx), R depends on theta only through the
residual r = u - x0 - tx z:  R = exp(-r^2 / sigma^2).  In the scaled
coordinates theta~ = diag(1, z_ref) theta the gradient and the Hessian are
both along phi~ = (1, z / z_ref), so
  * when 2 r^2 < sigma^2 the Hessian is negative along phi~, conjugate
    gradients end after one iteration with the exact Newton step along phi~,
    and the residual moves by  dr = -r sigma^2 / (sigma^2 - 2 r^2);
  * otherwise the first CG direction meets non-positive curvature and the
    step is one bandwidth along the scaled gradient: |dr| = sigma |phi~|,
    towards the hit;
  * the scaled step length is |dr| / |phi~|;
  * a step changes theta by (-dr) (1, z / z_ref^2) / |phi~|^2;
  * the Armijo test at step length alpha compares exp(-(r + alpha dr)^2 /
    sigma^2) with R + c1 alpha g.p, where g.p = (2 r R / sigma^2)(-dr).
`_reduce` below follows exactly that, in closed form, with no linear algebra:
it shares nothing with the oracle's CG, its 2 x 2 arithmetic or its response
sums.  The polish is switched off (n_polish = 0), so the oracle's per-seed
theta is the state after the steps.  Each case is chosen so that a flipped
Armijo inequality, a missing alpha in the sufficient-increase term, another
halving order, an off-by-one in the trial count or in the schedule, or a
shortcut threshold not scaled by sigma changes the outcome."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import oracle

Z = np.array([1.0, 2.0], np.float32)          # two planes; the hit sits on the first
ZREF = math.sqrt((1.0 + 4.0) / 2.0)           # RMS plane position
PHI2 = 1.0 + (1.0 / ZREF) ** 2                # |phi~|^2 for the hit's plane (z = 1)
DIR = np.array([1.0, 1.0 / ZREF ** 2])        # theta direction of a step: (1, z / z_ref^2)


def _event(u):
    return SimpleNamespace(meas_dim=1, plane_z=Z, event_offsets=np.array([0, 1], np.int64),
                           x=np.array([u], np.float32), y=None, plane=np.array([0], np.int32))


def _params(sigma, sigma_final=1.0, n_final=0, c1=0.25, trials=4, cap=100.0, small=0.0):
    return dict(sigma=list(sigma), sigma_final=sigma_final, n_final_steps=n_final, n_polish=0,
                ls_trials=trials, armijo_c1=c1, step_cap_sigmas=cap, small_step_sigmas=small,
                conv_tol=1.0, R0=0.5, d_merge=0.01, lattice_n=[1, 1], lattice_lo=[0.0, 0.0],
                lattice_hi=[1.0, 1.0], n_slope_steps=0)


def _run(u, P, seed=(0.0, 0.0)):
    ev = _event(u)
    ref = oracle.find_tracks(ev, P, seeds=np.array([seed], np.float64), seed_offsets=np.array([0, 1], np.int64))
    return ref["seed_theta"][0], int(ref["seed_flags"][0]), int(ref["seed_nreval"][0])


def _reduce(r, P):
    """The method on the one-hit problem, in the residual alone (see the module
    docstring).  Returns (final r, R-only evaluations, stalled, negative curvature)."""
    sched = list(P["sigma"]) + [P["sigma_final"]] * P["n_final_steps"]
    n_reval, stalled, neg_any = 0, False, False
    phin = math.sqrt(PHI2)
    for sig in sched:
        R = math.exp(-r * r / sig ** 2)
        neg = not (2.0 * r * r < sig * sig)
        if neg:
            dr = -math.copysign(sig * phin, r)
        else:
            dr = -r * sig * sig / (sig * sig - 2.0 * r * r)
        pn = abs(dr) / phin
        if pn > P["step_cap_sigmas"] * sig:
            dr *= P["step_cap_sigmas"] * sig / pn
            pn = P["step_cap_sigmas"] * sig
        neg_any |= neg
        if not neg and pn <= P["small_step_sigmas"] * sig:
            r += dr
            continue
        gp = (2.0 * r * R / sig ** 2) * (-dr)
        alpha, done = 1.0, False
        for _ in range(P["ls_trials"]):
            n_reval += 1
            rt = r + alpha * dr
            if math.exp(-rt * rt / sig ** 2) >= R + P["armijo_c1"] * alpha * gp:
                r, done = rt, True
                break
            alpha *= 0.5
        stalled |= not done
    return r, n_reval, stalled, neg_any


def _theta_of(u, r_final, seed=(0.0, 0.0)):
    r0 = float(np.float32(u)) - seed[0] - seed[1] * 1.0
    return np.array(seed) + (r0 - r_final) / PHI2 * DIR


def _check(u, P, n_reval, stalled, neg, theta=None):
    """The oracle against the scalar reduction, and against stated outcomes."""
    th, fl, nr = _run(u, P)
    r, nr_ref, st_ref, neg_ref = _reduce(float(np.float32(u)), P)
    assert (nr_ref, st_ref, neg_ref) == (n_reval, stalled, neg), "the case does not test what it states"
    assert nr == n_reval
    assert bool(fl & oracle.STALLED) == stalled
    assert bool(fl & oracle.NEGCURV) == neg
    np.testing.assert_allclose(th, _theta_of(u, r), rtol=1e-12, atol=1e-14)
    if theta is not None:
        np.testing.assert_allclose(th, theta, rtol=1e-12, atol=1e-14)
    return th


def test_full_newton_step_rejected_half_step_accepted():
    """r = 0.5, sigma = 1: the Newton step overshoots to r = -0.5, where R is
    unchanged, so alpha = 1 fails the sufficient-increase test; alpha = 1/2
    lands on the hit (R = 1).  With c1 = 0.4, R + c1 alpha g.p is 0.8995 at
    alpha = 1/2 but 1.0903 without the alpha, so a missing alpha stalls."""
    P = _params([1.0], c1=0.4)
    th = _check(0.5, P, n_reval=2, stalled=False, neg=False, theta=[0.5 / PHI2, 0.5 / PHI2 / ZREF ** 2])
    # the line now passes through the hit: x0 + tx z = u
    assert th[0] + th[1] * 1.0 == pytest.approx(0.5, abs=1e-15)


def test_fourth_step_length_accepted():
    """c1 = 0.87: alpha = 1, 1/2, 1/4 fail and alpha = 1/8 passes (n_reval 4);
    with three trials the same search stalls and theta stays at the seed."""
    _check(0.5, _params([1.0], c1=0.87), n_reval=4, stalled=False, neg=False,
           theta=[0.125 * 1.0 / PHI2, 0.125 * 1.0 / PHI2 / ZREF ** 2])
    _check(0.5, _params([1.0], c1=0.87, trials=3), n_reval=3, stalled=True, neg=False, theta=[0.0, 0.0])


@pytest.mark.parametrize("trials", [1, 2, 4])
def test_no_step_length_accepted(trials):
    """c1 = 0.99: no alpha in (1, 1/2, 1/4, 1/8) gives enough increase; theta is
    unchanged, the seed is flagged stalled and every trial was evaluated."""
    _check(0.5, _params([1.0], c1=0.99, trials=trials), n_reval=trials, stalled=True, neg=False,
           theta=[0.0, 0.0])


def test_short_newton_step_taken_without_search():
    """sigma = 2, r = 0.5: the Newton step's scaled length is 0.4830.  A threshold
    of 0.3 sigma = 0.6 takes it directly (no R evaluation); 0.2 sigma = 0.4 sends
    it through the line search, which accepts alpha = 1.  Same theta both ways."""
    a = _check(0.5, _params([2.0], small=0.3), n_reval=0, stalled=False, neg=False)
    b = _check(0.5, _params([2.0], small=0.2), n_reval=1, stalled=False, neg=False)
    np.testing.assert_array_equal(a, b)


def test_shortcut_never_applies_under_negative_curvature():
    """Far from the hit (r = 10, sigma = 2) the step is a normalised-gradient step
    of one bandwidth; even a huge shortcut threshold leaves it to the search."""
    _check(10.0, _params([2.0], small=100.0), n_reval=1, stalled=False, neg=True,
           theta=[2.0 / math.sqrt(PHI2), 2.0 / math.sqrt(PHI2) / ZREF ** 2])


def test_step_cap():
    """cap 0.5: the normalised-gradient step of one bandwidth is cut to half a
    bandwidth in scaled units."""
    _check(10.0, _params([2.0], cap=0.5), n_reval=1, stalled=False, neg=True,
           theta=[1.0 / math.sqrt(PHI2), 1.0 / math.sqrt(PHI2) / ZREF ** 2])


def test_schedule_order_stages_then_final():
    """Stages sigma = (2, 1), then two steps at sigma_final = 0.2.  From
    u = 0.25 + 2 |phi~| the first step (convex region at sigma 2) moves one
    bandwidth to r = 0.25, the second (concave at sigma 1) is a Newton step to
    r = -1/28, the final steps are Newton steps at 0.2.  Taking the stages in
    the other order, or sigma_final one step early or late, ends elsewhere."""
    u = float(np.float32(0.25 + 2.0 * math.sqrt(PHI2)))
    P = _params([2.0, 1.0], sigma_final=0.2, n_final=2, c1=1e-4)
    r1 = u - 2.0 * math.sqrt(PHI2)
    r2 = r1 - r1 * 1.0 / (1.0 - 2.0 * r1 * r1)  # r + dr, dr = -r sigma^2 / (sigma^2 - 2 r^2)
    assert r2 == pytest.approx(-1.0 / 28.0, rel=1e-6)
    th = _check(u, P, n_reval=4, stalled=False, neg=True)
    # the same stages in another order, or another count at sigma_final, end
    # elsewhere (one extra Newton step at 0.2 still moves r by 5e-7)
    for other in (_params([1.0, 2.0], sigma_final=0.2, n_final=2, c1=1e-4),
                  _params([2.0, 1.0], sigma_final=0.2, n_final=1, c1=1e-4),
                  _params([2.0, 1.0, 0.2], sigma_final=0.2, n_final=2, c1=1e-4),
                  _params([2.0, 1.0], sigma_final=1.0, n_final=2, c1=1e-4)):
        r_o = _reduce(u, other)[0]
        assert np.abs(_theta_of(u, r_o) - th).max() > 1e-9  # far outside the 1e-12 bar above
