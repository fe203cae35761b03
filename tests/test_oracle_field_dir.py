"""Pins of the applied-field direction e_H in the oracle (Sec. II.1 with the field
along a unit vector instead of x; loop, area and Eq. 6 take components along e_H).

* Rotation invariance: rotating positions, axes and the field direction together
  leaves every scalar of the run unchanged: loop, per-particle areas, Eq. 6 field
  differences (interacting assembly at T > 0, the same Philox draws), and the
  mean-magnetisation loop.
* Easy axis along the field (both along z, T = 0): the square loop with its exact area,
  as for x.
* Hard axis (axes along x, field along z, T = 0): the moment follows the closed form
  m . z = clip(H / H_K, -1, 1), so the recorded loop and area are those of that curve.
"""
import numpy as np

from oracle import kmc, master
from paper_1407_2737_amd import workloads as W


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def test_rotation_invariance_interacting_T300():
    n = 40
    pos = W.place_random(n, 45e-9, 12e-9, 3)
    axes = W.axes_random_3d(n, 4)
    p = kmc.Params(T=300.0, mu0Hmax=0.03, steps_per_period=200, n_periods=2, n_discard=1)
    Q = _rotation(7)
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-15) and np.linalg.det(Q) > 0
    r0 = kmc.simulate(pos, axes, p, seed=11)
    p1 = kmc.Params(**{**p.__dict__, "field_dir": tuple(Q[:, 0] * 2.5)})  # not normalised
    r1 = kmc.simulate(pos @ Q.T, axes @ Q.T, p1, seed=11)
    assert r0.jumps > 0 and r1.jumps == r0.jumps
    assert np.abs(r1.M - r0.M).max() < 1e-9 * p.Ms
    assert np.abs(r1.area_per_np - r0.area_per_np).max() < 1e-9 * np.abs(r0.area_per_np).max()
    assert np.abs(r1.dhdip_per_np - r0.dhdip_per_np).max() < 1e-9 * np.abs(r0.dhdip_per_np).max()
    assert np.abs(r1.m_final - r0.m_final @ Q.T).max() < 1e-9


def test_rotation_invariance_mean_loop():
    n = 50
    axes = W.axes_random_3d(n, 8)
    p = kmc.Params(T=300.0, mu0Hmax=0.03, steps_per_period=200, n_periods=2, n_discard=1,
                   interactions=0)
    Q = _rotation(9)
    H0, M0, A0 = master.mean_loop(axes, p)
    p1 = kmc.Params(**{**p.__dict__, "field_dir": tuple(Q[:, 0])})
    H1, M1, A1 = master.mean_loop(axes @ Q.T, p1)
    assert np.array_equal(H0, H1)
    assert np.abs(M1 - M0).max() < 1e-9 * p.Ms
    assert abs(A1 - A0) < 1e-9 * abs(A0)


def test_square_loop_along_z():
    p = kmc.Params(T=0.0, mu0Hmax=0.1, Ms=4e5, Keff=1.3e4, steps_per_period=400, n_periods=2,
                   n_discard=1, interactions=0, field_dir=(0.0, 0.0, 1.0))
    BK = 2 * p.Keff / p.Ms
    r = kmc.simulate(np.zeros((1, 3)), np.array([[0.0, 0.0, -1.0]]), p, seed=1)
    H, S = r.H, p.steps_per_period
    kd = next(k for k in range(S) if H[k] <= -BK)
    ku = next(k for k in range(S // 2, S) if H[k] >= BK)
    want = np.where((np.arange(S) >= kd) & (np.arange(S) < ku), -p.Ms, p.Ms)
    assert np.array_equal(r.M[0], want)
    area = 2 * p.Ms * (abs(H[kd]) + H[ku])
    assert abs(r.area - area) < 1e-9 * area


def test_hard_axis_follows_closed_form():
    p = kmc.Params(T=0.0, mu0Hmax=0.1, Ms=4e5, Keff=1.3e4, steps_per_period=400, n_periods=2,
                   n_discard=1, interactions=0, field_dir=(0.0, 0.0, 1.0))
    BK = 2 * p.Keff / p.Ms
    axes = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    r = kmc.simulate(np.zeros((2, 3)), axes, p, seed=1)
    S = p.steps_per_period
    H = p.mu0Hmax * np.cos(2 * np.pi * np.arange(-1, S) / S)
    mz = np.clip(H / BK, -1.0, 1.0)
    assert np.abs(r.M[0] - p.Ms * mz[1:]).max() < 1e-9 * p.Ms
    # area of the reversible curve sampled at the step fields (left-endpoint rule)
    area = p.Ms * np.sum(H[1:] * (mz[1:] - mz[:-1]))
    assert abs(r.area - area) < 1e-9 * p.Ms * BK
