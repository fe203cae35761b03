"""Quasi-static (T = 0) Stoner-Wohlfarth major loop of randomly oriented particles by
one-dimensional quadrature over the axis angle psi (Stoner and Wohlfarth, 1948).

Independent of the kMC step code: it uses only the closed forms of the model.

* Switching field of a particle whose axis makes angle psi with the field:
  h_sw(psi) = (cos^(2/3) psi + sin^(2/3) psi)^(-3/2).
* At the switching field the vanishing minimum is the double root theta* of e'
  with (hx, hy) = (-cos^3 theta*, sin^3 theta*) (the point of tangency on the astroid).
* The loop area of one particle is twice the energy it dissipates in one jump,
  2 K (e(theta*) - e(theta_land)); reversible rotation dissipates nothing.
* Remanence on the major loop is M_S <|cos psi|> = M_S / 2.

The paper quotes A / K_eff = 2 for randomly oriented, non-interacting particles
(Sec. III.2.c), which this reproduces as a pin.
"""
import numpy as np
from scipy import integrate, optimize


def h_switch(psi):
    c = np.abs(np.cos(psi)) ** (2.0 / 3.0)
    s = np.abs(np.sin(psi)) ** (2.0 / 3.0)
    return (c + s) ** -1.5


def _e(theta, hx, hy):
    return np.sin(theta) ** 2 - 2.0 * (hx * np.cos(theta) + hy * np.sin(theta))


def _g(theta, hx, hy):
    return np.sin(theta) * np.cos(theta) + hx * np.sin(theta) - hy * np.cos(theta)


def jump_energy(psi):
    """Energy drop (units of K V) when the descending branch switches, axis at psi in
    [0, pi/2] from +x. theta is measured from the axis in the (axis, x) plane, so a
    field h along x has components (h cos psi, -h sin psi)."""
    hs = h_switch(psi)
    hx, hy = -hs * np.cos(psi), hs * np.sin(psi)     # h = -hs along x
    # double root: tan^3 theta* = -hy/hx with cos theta* of sign -hx, sin of sign hy
    ct = np.cbrt(-hx)
    st = np.cbrt(hy)
    th_star = np.arctan2(st, ct)
    # the remaining minimum lies between the axis end nearest the field (theta = pi)
    # and the field direction (theta = pi - psi)
    a, b = np.pi - psi, np.pi
    if psi == 0.0:
        th_land = np.pi
    else:
        th_land = optimize.brentq(_g, a, b, args=(hx, hy), xtol=1e-15)
    return _e(th_star, hx, hy) - _e(th_land, hx, hy)


def random_axis_area_over_K(hmax: float = np.inf):
    """<A>/K for axes uniform on the sphere; particles with h_sw(psi) > hmax never switch."""
    def f(psi):
        if h_switch(psi) > hmax:
            return 0.0
        return 2.0 * jump_energy(psi) * np.sin(psi)
    val, _ = integrate.quad(f, 0.0, np.pi / 2, limit=200, epsabs=1e-12, epsrel=1e-12)
    return val


def branch_mx(h, psi):
    """m_x on the descending branch at reduced field h (from +saturation), axis psi."""
    hx, hy = h * np.cos(psi), -h * np.sin(psi)
    if h >= 0 or -h < h_switch(psi):
        # still in the well that started near theta = 0 (between -psi and 0 side)
        lo, hi = -np.pi / 2, np.pi / 2
        ts = np.linspace(lo, hi, 4001)
        gv = _g(ts, hx, hy)
        idx = np.nonzero((gv[:-1] < 0) & (gv[1:] >= 0))[0]
        cands = [optimize.brentq(_g, ts[i], ts[i + 1], args=(hx, hy), xtol=1e-15) for i in idx]
        th = min(cands, key=lambda t: abs(t))
    else:
        th = optimize.brentq(_g, np.pi - psi, np.pi, args=(hx, hy), xtol=1e-15)
    return np.cos(th - (-psi))


def random_axis_coercivity():
    """Reduced coercive field h_c of the random-axis descending branch."""
    def M(h):
        pts = []
        if -h > 0.5:          # the switched set is an interval around psi = pi/4
            pts = [optimize.brentq(lambda p: h_switch(p) + h, 0.0, np.pi / 4),
                   optimize.brentq(lambda p: h_switch(p) + h, np.pi / 4, np.pi / 2)]
        val, _ = integrate.quad(lambda p: branch_mx(h, p) * np.sin(p), 0.0, np.pi / 2,
                                limit=200, points=pts or None)
        return val
    return -optimize.brentq(M, -0.6, -0.4, xtol=1e-7)
