"""Pins of whole hysteresis loops produced by the oracle (Sec. II.1, Sec. II.3,
Sec. III.1, Sec. III.2.c).

* T = 0, one particle with its axis along the field: square loop that switches at
  the first sampled |H_k| >= H_K = 2K/(mu0 M_S), area 2 M_S (|B_k-| + B_k+).
* T = 0, non-interacting particles with axes spread uniformly over the sphere
  (stratified in cos psi): area / K, remanence and coercive field equal the
  Stoner-Wohlfarth quadrature (A/K = 1.977, the paper's "2"; M_r = M_S/2;
  h_c = 0.482).
* T > 0, no interactions: the kMC loop averaged over particles equals the
  deterministic mean-magnetisation loop (the paper's own validation, Fig. 1(c)-(d)).
* Two interacting particles: the sampled mean moment after a few steps equals the
  exact expectation obtained by enumerating every jump branch (brute force)."""
import itertools

import numpy as np
import pytest

from oracle import kmc, master, swloop


def test_aligned_square_loop_T0():
    p = kmc.Params(T=0.0, mu0Hmax=0.1, Ms=4e5, Keff=1.3e4, steps_per_period=400,
                   n_periods=2, n_discard=1, interactions=0)
    BK = 2 * p.Keff / p.Ms
    assert abs(BK - 0.065) < 1e-15             # 65 mT for this material
    axes = np.array([[1.0, 0.0, 0.0]])
    r = kmc.simulate(np.zeros((1, 3)), axes, p, seed=1)
    H = r.H
    S = p.steps_per_period
    kd = next(k for k in range(S) if H[k] <= -BK)
    ku = next(k for k in range(S // 2, S) if H[k] >= BK)
    want = np.where((np.arange(S) >= kd) & (np.arange(S) < ku), -p.Ms, p.Ms)
    assert np.array_equal(r.M[0], want)
    area = 2 * p.Ms * (abs(H[kd]) + H[ku])
    assert abs(r.area - area) < 1e-9 * area


def _stratified_axes(n):
    c = (np.arange(n) + 0.5) / n                 # cos psi uniform on (0, 1)
    az = np.arange(n) * np.pi * (3 - np.sqrt(5))  # golden-angle azimuths
    s = np.sqrt(1 - c * c)
    return np.stack([c, s * np.cos(az), s * np.sin(az)], axis=1)


def test_random_axes_T0_matches_stoner_wohlfarth():
    n = 160
    # two periods, first discarded: the first one starts with moments on their axes,
    # so it is not a closed loop (Sec. III.1)
    p = kmc.Params(T=0.0, mu0Hmax=1.2 * 0.065, Ms=4e5, Keff=1.3e4, steps_per_period=2000,
                   n_periods=2, n_discard=1, interactions=0)
    axes = _stratified_axes(n)
    r = kmc.simulate(np.zeros((n, 3)), axes, p, seed=1)
    A_over_K = r.area / p.Keff
    ref = swloop.random_axis_area_over_K()
    assert abs(ref - 1.9766) < 1e-3 and round(ref) == 2      # the paper's A/K = 2
    assert abs(A_over_K - ref) < 0.01 * ref
    # remanence where the field crosses zero on the way down
    S = p.steps_per_period
    Mr = 0.5 * (r.M[0][S // 4 - 1] + r.M[0][S // 4]) / p.Ms
    assert abs(Mr - 0.5) < 0.01
    # coercive field: interpolate the descending branch through M = 0
    M, H = r.M[0][: S // 2], r.H[: S // 2]
    k = int(np.nonzero(M < 0)[0][0])
    hc = -(H[k - 1] + (H[k] - H[k - 1]) * M[k - 1] / (M[k - 1] - M[k])) / 0.065
    hc_ref = swloop.random_axis_coercivity()
    assert abs(hc_ref - 0.482) < 1e-3
    assert abs(hc - hc_ref) < 0.015 * hc_ref


@pytest.mark.parametrize("d,K,H,n", [(12e-9, 1.3e4, 0.02, 800), (20e-9, 1.3e4, 0.04, 400)])
def test_kmc_matches_mean_magnetisation_loop(d, K, H, n):
    p = kmc.Params(T=300.0, d=d, Keff=K, mu0Hmax=H, Ms=4e5, steps_per_period=400,
                   n_periods=2, n_discard=1, interactions=0)
    rng = np.random.default_rng(21)
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    r = kmc.simulate(np.zeros((n, 3)), axes, p, seed=77)
    Hm, Mm, Am = master.mean_loop(axes, p)
    se = r.area_per_np.std(ddof=1) / np.sqrt(n)
    assert abs(r.area - Am) < 4 * se + 1e-9 * abs(Am), (r.area, Am, se)
    # loop points: per-step standard error of the mean of m_x is at most M_S/sqrt(n)
    assert np.max(np.abs(r.M[0] - Mm[0])) < 5 * p.Ms / np.sqrt(n)


def _enumerate(pos, axes, m0, p, steps):
    """Exact E[<m_x>] after ``steps`` steps by enumerating all jump branches."""
    leaves = [(1.0, m0)]
    for k in range(steps):
        nxt = []
        for w, m in leaves:
            _, info = kmc.step(pos, axes, m, k, p, seed=0, stream=0)
            opts = []
            for i in range(m.shape[0]):
                th = [(1.0 - info.P[i], info.theta_c[i])]
                if info.two[i] and info.P[i] > 0:
                    th.append((info.P[i], info.theta_o[i]))
                opts.append([(q, np.cos(t) * axes[i] + np.sin(t) * info.u2[i]) for q, t in th])
            for combo in itertools.product(*opts):
                q = np.prod([c[0] for c in combo])
                nxt.append((w * q, np.array([c[1] for c in combo])))
        leaves = nxt
    return sum(w * m[:, 0].mean() for w, m in leaves), sum(w for w, _ in leaves)


def test_two_particles_brute_force():
    d = 8e-9
    p = kmc.Params(T=300.0, d=d, Keff=1.3e4, Ms=4e5, mu0Hmax=0.004, dt_override=1e-10,
                   interactions=1)
    pos = np.array([[0.0, 0.0, 0.0], [1.05 * d * 0.6, 1.05 * d * 0.8, 0.0]])
    axes = np.array([[1.0, 0.0, 0.0], [0.6, 0.0, 0.8]])
    m0 = kmc.initial_moments(axes)
    steps = 3
    want, wsum = _enumerate(pos, axes, m0, p, steps)
    assert abs(wsum - 1.0) < 1e-12
    R = 3000
    vals = np.empty(R)
    for r in range(R):
        m = m0
        for k in range(steps):
            m, _ = kmc.step(pos, axes, m, k, p, seed=12345, stream=r)
        vals[r] = m[:, 0].mean()
    se = vals.std(ddof=1) / np.sqrt(R)
    assert se > 0.005                      # the branches really differ
    assert abs(vals.mean() - want) < 4 * se, (vals.mean(), want, se)


def test_scan200_mode_T0_loop_matches_stoner_wohlfarth():
    """The paper-literal extremum scan (step iv with 200 grid points) loses a close
    saddle/minimum pair only within about 1e-4 of the switching field, so its T = 0
    loop over random axes still gives the Stoner-Wohlfarth area and coercive field."""
    n = 160
    p = kmc.Params(T=0.0, mu0Hmax=1.2 * 0.065, Ms=4e5, Keff=1.3e4, steps_per_period=2000,
                   n_periods=2, n_discard=1, interactions=0, extrema_mode=1)
    r = kmc.simulate(np.zeros((n, 3)), _stratified_axes(n), p, seed=1)
    ref = swloop.random_axis_area_over_K()
    assert abs(r.area / p.Keff - ref) < 0.01 * ref
    p0 = kmc.Params(**{**p.__dict__, "extrema_mode": 0})
    r0 = kmc.simulate(np.zeros((n, 3)), _stratified_axes(n), p0, seed=1)
    # a particle switches at most one field sample earlier than with the exact search
    dM = np.abs(r.M[0] - r0.M[0])
    assert np.count_nonzero(dM) <= 2 * 2 * n
