"""Pins of the switching probability (Eqs. 3-5, Sec. II.1 steps vi-vii).

Fig. 1(b): with nu1 = 1 Hz and nu2 = 0.2 Hz the occupation of the first well tends to
nu2/(nu1+nu2) = 0.166..., the relaxation time is 1/(nu1+nu2) and the initial slope
is nu2. In a static field the two-state chain of Eq. 5 has the Boltzmann ratio
exp(-(E_c - E_o)/kT) as stationary occupation for any step length, which the
single-rate form 1 - exp(-dt/tau) does not have."""
import numpy as np

from oracle import kmc


def test_fig1b_numbers():
    nu1, nu2 = 1.0, 0.2
    # start in well 2 (rate out nu2); a = -ln(nu/nu0) with nu0 = 1 Hz, nu0 dt = t
    a_c, a_o = -np.log(nu2), -np.log(nu1)
    P_inf = kmc.transition_probability(a_c, a_o, 1e6)
    assert abs(P_inf - 0.2 / 1.2) < 1e-15
    assert abs(P_inf - 0.166) < 1e-3          # value printed in the caption
    tau = 1.0 / (nu1 + nu2)
    assert abs(kmc.transition_probability(a_c, a_o, tau) - P_inf * (1 - np.exp(-1))) < 1e-15
    t = 1e-7
    assert abs(kmc.transition_probability(a_c, a_o, t) / t - nu2) < 1e-6
    # symmetric wells: relaxation toward 1/2
    assert abs(kmc.transition_probability(3.0, 3.0, 1e9) - 0.5) < 1e-15
    # no overflow for huge barriers
    assert kmc.transition_probability(5000.0, 4000.0, 50.0) == 0.0


def _static_chain(p, hx_T, steps, n=3000, seed=99):
    axes = np.tile([1.0, 0.0, 0.0], (n, 1))
    pos = np.zeros((n, 3))
    m = kmc.initial_moments(axes)
    for k in range(steps):
        m, info = kmc.step(pos, axes, m, k, p, seed, 0)
    return m, info


def test_boltzmann_occupation_any_dt():
    # static field along the axis, non-interacting: wells at 0 and pi,
    # e(0) = -2h, e(pi) = +2h, so P(pi)/P(0) = exp(-beta 4 h)
    for nu0dt in (0.5, 3.0, 50.0):
        p = kmc.Params(Keff=1.3e4, Ms=4e5, d=8e-9, T=300.0, mu0Hmax=0.004, interactions=0,
                       dt_override=nu0dt * 1e-10)
        dv = kmc.derived(p)
        h = p.mu0Hmax / dv["BK"]
        # relaxation per step is exp(-nu0 dt (e^-a1 + e^-a2)); run 8 relaxation times
        a1 = dv["beta"] * (1 + h) ** 2
        relax = 1.0 / (nu0dt * (np.exp(-a1) + np.exp(-dv["beta"] * (1 - h) ** 2)))
        steps = int(max(6, 8 * relax))
        assert steps <= 40
        m, info = _static_chain(p, p.mu0Hmax, steps)
        frac_pi = np.mean(m[:, 0] < 0)
        want = 1.0 / (1.0 + np.exp(dv["beta"] * 4 * h))
        se = np.sqrt(want * (1 - want) / m.shape[0])
        assert abs(frac_pi - want) < 4.5 * se, (nu0dt, frac_pi, want)


def test_single_rate_form_is_not_boltzmann_at_large_dt():
    p = kmc.Params(Keff=1.3e4, Ms=4e5, d=8e-9, T=300.0, mu0Hmax=0.004, interactions=0,
                   dt_override=50 * 1e-10, prob_form=1)
    dv = kmc.derived(p)
    h = p.mu0Hmax / dv["BK"]
    m, info = _static_chain(p, p.mu0Hmax, 10)
    frac_pi = np.mean(m[:, 0] < 0)
    want = 1.0 / (1.0 + np.exp(dv["beta"] * 4 * h))
    se = np.sqrt(want * (1 - want) / m.shape[0])
    assert abs(frac_pi - want) > 10 * se


def test_zero_temperature_never_jumps():
    p = kmc.Params(T=0.0, interactions=0, mu0Hmax=0.03, steps_per_period=200)
    rng = np.random.default_rng(1)
    axes = rng.normal(size=(300, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    m = kmc.initial_moments(axes)
    for k in range(60):
        m, info = kmc.step(np.zeros((300, 3)), axes, m, k, p, 1, 0)
        assert not info.jump.any()


def test_sar_conversion():
    # Sec. III.2.a: 10^4 J/m^3 at 100 kHz and rho = 5200 kg/m^3 is 192 W/g
    sar = kmc.sar_from_area(1e4, 1e5, 5200.0)
    assert abs(sar / 1000.0 - 192.3) < 0.05
    assert round(sar / 1000.0) == 192
