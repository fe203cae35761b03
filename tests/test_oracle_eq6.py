"""Eq. 6 (Sec. III.3): Delta-_Hdip = mu0 H_dip^x(+mu0 Hmax) - mu0 H_dip^x(-mu0 Hmax) per
particle, pinned by closed forms.

With easy axes along the field, a 1 T field and mu0 H_K = 5 mT at T = 0, every moment
is exactly +x at the +Hmax step and -x at the -Hmax step (eight steps per period, so
the moments have followed the field before those steps). A contact pair along x then
sees the on-axis dipole field mu0 M_S/12 at +Hmax and its negative at -Hmax:
Delta = mu0 M_S/6; a broadside pair sees -mu0 M_S/24 and +mu0 M_S/24: Delta =
-mu0 M_S/12. Without interactions Delta = 0."""
import numpy as np
import pytest

from oracle import kmc

D = 12e-9
MS = 4e5
MU0MS = kmc.MU0 * MS


def _run(pos, interactions=1, periods=3):
    n = pos.shape[0]
    axes = np.tile([1.0, 0.0, 0.0], (n, 1))
    p = kmc.Params(Ms=MS, Keff=1e3, d=D, T=0.0, mu0Hmax=1.0, steps_per_period=8,
                   n_periods=periods, n_discard=1, interactions=interactions)
    return kmc.simulate(pos, axes, p, seed=1)


def test_pair_along_field():
    r = _run(np.array([[0.0, 0, 0], [D, 0, 0]]))
    assert np.allclose(r.dhdip_per_np, MU0MS / 6, rtol=1e-12, atol=0)


def test_pair_broadside():
    r = _run(np.array([[0.0, 0, 0], [0, D, 0]]))
    assert np.allclose(r.dhdip_per_np, -MU0MS / 12, rtol=1e-12, atol=0)
    r = _run(np.array([[0.0, 0, 0], [0, 0, 2 * D]]))       # r^-3 scaling
    assert np.allclose(r.dhdip_per_np, -MU0MS / 96, rtol=1e-12, atol=0)


def test_no_interactions_is_zero():
    r = _run(np.array([[0.0, 0, 0], [D, 0, 0], [0, 2 * D, 0]]), interactions=0)
    assert np.all(r.dhdip_per_np == 0.0)


@pytest.mark.parametrize("periods", [2, 4])
def test_line_of_three_superposes(periods):
    """Middle of three along x: two contact neighbours, 2 x mu0 M_S/6; ends: one at d and
    one at 2d, (1 + 1/8) mu0 M_S/6; the mean over kept periods does not depend on how
    many are kept."""
    r = _run(np.array([[-D, 0, 0], [0.0, 0, 0], [D, 0, 0]]), periods=periods)
    want = np.array([1.125, 2.0, 1.125]) * MU0MS / 6
    assert np.allclose(r.dhdip_per_np, want, rtol=1e-12, atol=0)
