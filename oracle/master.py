"""Deterministic mean-magnetisation loop of non-interacting particles (the paper's
validation method, Sec. II.3): instead of one sampled well per particle, the
probability of occupying each well is carried, and the loop is the
probability-weighted moment, i.e. the loop of an infinite number of particles.

Per particle the state is at most two weighted moment vectors. Each step every
weighted vector is projected into the new working plane and falls into a minimum
(steps iii-v); each minimum's weight is then moved across the barrier with the exact
two-state transition of Eq. 5 (steps vi-vii): the weight w_c in well c sends
w_c P(c->o) to well o. With T = 0 no weight moves.

The expected value of the kMC oracle's loop (kmc.simulate with interactions off,
averaged over independent Philox streams) equals this loop, which is the comparison
the paper makes in Fig. 1(c)-(d).
"""
import numpy as np

from . import kmc
from . import sw


def _fall(B, axes, mvec, BK):
    u2, hx, hy, theta0 = kmc.working_plane(B, axes, mvec, BK)
    theta, is_min, count = sw.stationary_points(hx, hy)
    th_c, e_c, th_o, e_o, e3, two = sw.classify(theta0, theta, is_min, count, hx, hy)
    return u2, th_c, e_c, th_o, e_o, e3, two


def mean_loop(axes: np.ndarray, p: kmc.Params):
    """Returns (H (S,), M (n_kept, S) expected M_S <m . e_H>, expected area J/m^3)."""
    if p.interactions:
        raise ValueError("the mean-magnetisation loop is defined for non-interacting particles")
    dv = kmc.derived(p)
    n = axes.shape[0]
    S = p.steps_per_period
    total = p.n_periods * S
    kept0 = p.n_discard * S
    n_kept = p.n_periods - p.n_discard
    eH = kmc.field_unit(p)
    mA = kmc.initial_moments(axes, eH)
    wA = np.ones(n)
    mB = mA.copy()
    wB = np.zeros(n)
    Mrec = np.zeros((n_kept, S))
    Hrec = np.array([kmc.applied_field(k, p) for k in range(S)])
    area = 0.0
    mx_prev = (wA * (mA @ eH) + wB * (mB @ eH)).mean()
    for k in range(total):
        Bx = kmc.applied_field(k, p)
        B = np.zeros((n, 3)) + Bx * eH[None, :]
        uA, thcA, ecA, thoA, eoA, e3A, two = _fall(B, axes, mA, dv["BK"])
        uB, thcB, ecB, thoB, eoB, e3B, _ = _fall(B, axes, mB, dv["BK"])
        # both weighted vectors live in the same plane unless it is degenerate; the
        # minima are the same two angles, so weights are pooled by minimum angle
        w1 = np.zeros(n)
        w2 = np.zeros(n)
        t1 = thcA.copy()
        t2 = thoA.copy()
        w1 += wA
        sameB = np.isclose(thcB, t1, rtol=0, atol=1e-9)
        w1 += np.where(sameB, wB, 0.0)
        w2 += np.where(sameB, 0.0, wB)
        if p.T > 0:
            a1 = dv["beta"] * (e3A - ecA)
            a2 = dv["beta"] * (e3A - eoA)
            P12 = np.where(two, kmc.transition_probability(np.where(two, a1, 0.0),
                                                           np.where(two, a2, 0.0),
                                                           dv["nu0dt"], p.prob_form), 0.0)
            P21 = np.where(two, kmc.transition_probability(np.where(two, a2, 0.0),
                                                           np.where(two, a1, 0.0),
                                                           dv["nu0dt"], p.prob_form), 0.0)
            n1 = w1 * (1.0 - P12) + w2 * P21
            n2 = w2 * (1.0 - P21) + w1 * P12
            w1, w2 = n1, n2
        # one minimum left: all weight is in it
        w1 = np.where(two, w1, 1.0)
        w2 = np.where(two, w2, 0.0)
        mA = np.cos(t1)[:, None] * axes + np.sin(t1)[:, None] * uA
        mB = np.cos(t2)[:, None] * axes + np.sin(t2)[:, None] * uA
        wA, wB = w1, w2
        mx = (wA * (mA @ eH) + wB * (mB @ eH)).mean()
        if k >= kept0:
            area += p.Ms * Bx * (mx - mx_prev)
            Mrec[(k - kept0) // S, k % S] = p.Ms * mx
        mx_prev = mx
    return Hrec, Mrec, area / n_kept
