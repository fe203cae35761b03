"""The oracle against the numbers the paper prints (tests/golden/paper_values.txt, each
line citing its passage): the Fig. 1(b) occupation limit from Eq. 5, the area-to-SAR
conversion of Sec. III.2.a, the random-axis Stoner-Wohlfarth loop area of the dilute
limit, and the amplitude that keeps mu0 Hmax / K_eff fixed."""
import os

import numpy as np

from oracle import kmc, swloop

HERE = os.path.dirname(os.path.abspath(__file__))


def _values():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_values.txt")) as f:
        for line in f:
            body = line.split("#", 1)[0].split()
            if len(body) == 4:
                out[body[0]] = (float(body[1]), float(body[2]), body[3])
    return out


V = _values()


def _close(name, x):
    # cut: the printed value is x cut to its last digit, v <= x < v + unit;
    # round: x rounded to that digit, |x - v| <= unit / 2
    v, unit, mode = V[name]
    if mode == "cut":
        assert v - 1e-12 <= x < v + unit, (name, x, v, unit)
    else:
        assert abs(x - v) <= 0.5 * unit, (name, x, v, unit)


def test_fig1b_occupation_limit():
    # well 2 left at nu2, well 1 at nu1; after a long time the occupation of well 1 is
    # P(2 -> 1) over a step much longer than 1/(nu1 + nu2)
    a_c, a_o = -np.log(0.2), -np.log(1.0)     # nu0 = 1 Hz, so a = -ln(nu / nu0)
    _close("fig1b_p_inf", kmc.transition_probability(a_c, a_o, 1e6))


def test_sar_conversion():
    _close("sar_W_per_g_at_1e4", kmc.sar_from_area(1e4, 1e5, 5200.0) / 1e3)


def test_dilute_random_axis_area():
    _close("area_over_K_dilute", swloop.random_axis_area_over_K())


def test_constant_field_to_anisotropy_ratio():
    _close("mu0Hmax_at_K6000_mT", 40.0 * 6000.0 / 13000.0)
