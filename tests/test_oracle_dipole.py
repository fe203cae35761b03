"""Pins of Eq. 1 (exact dipolar field, Sec. II.1) in the oracle.

Closed forms: two particles at contact distance d give mu0 M_S / 12 along their axis
(2C/d^3 with C = mu0 M_S V / 4 pi and V = pi d^3 / 6) and -mu0 M_S / 24 broadside.
Invariants: the field at the centre of a cubic-lattice ball with uniform moments is
zero by cubic symmetry; the interaction is linear in the moments and reciprocal
(sum_i m_i . B_i[m'] = sum_i m'_i . B_i[m])."""
import math

import numpy as np

from oracle import kmc

MS = 4.0e5
D = 12e-9


def _C(d=D, ms=MS):
    return kmc.MU0 * ms * (np.pi * d ** 3 / 6) / (4 * np.pi)


def test_two_particles_on_axis_and_broadside():
    pos = np.array([[0.0, 0.0, 0.0], [D, 0.0, 0.0]])
    m = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    B = kmc.dipolar_field(pos, m, _C())
    assert np.allclose(B[0], [kmc.MU0 * MS / 12, 0, 0], rtol=1e-14, atol=0)
    assert np.allclose(B[1], [kmc.MU0 * MS / 12, 0, 0], rtol=1e-14, atol=0)
    assert abs(kmc.MU0 * MS / 12 - 0.041887902) < 1e-9         # 41.9 mT at M_S = 4e5 A/m
    m = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    B = kmc.dipolar_field(pos, m, _C())
    assert np.allclose(B[0], [0, 0, -kmc.MU0 * MS / 24], rtol=1e-14, atol=0)
    # r^-3 scaling and direction along an arbitrary line
    u = np.array([0.3, -0.5, 0.81])
    u /= np.linalg.norm(u)
    pos = np.array([[1e-9, 2e-9, -3e-9], [1e-9, 2e-9, -3e-9]]) + np.array([[0, 0, 0], 2.5 * D * u])
    m = np.array([[0, 0, 1.0], u])
    B = kmc.dipolar_field(pos, m, _C())
    assert np.allclose(B[0], 2 * _C() / (2.5 * D) ** 3 * u, rtol=1e-13, atol=0)


def test_cubic_lattice_centre_is_zero():
    a = 1.7 * D
    g = np.arange(-6, 7) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    P = P[np.linalg.norm(P, axis=1) <= 6 * a]
    centre = int(np.argmin(np.linalg.norm(P, axis=1)))
    for mv in ([0, 0, 1.0], [0.6, 0.0, 0.8], [1 / np.sqrt(3)] * 3):
        m = np.tile(np.array(mv), (P.shape[0], 1))
        B = kmc.dipolar_field(P, m, _C())
        scale = _C() / a ** 3
        assert np.max(np.abs(B[centre])) < 1e-12 * scale
        # off-centre particles do feel a field
        assert np.max(np.abs(B)) > 0.1 * scale


def test_linearity_and_reciprocity():
    rng = np.random.default_rng(3)
    n = 40
    pos = rng.uniform(-100e-9, 100e-9, size=(n, 3))
    m1 = rng.normal(size=(n, 3))
    m2 = rng.normal(size=(n, 3))
    C = _C()
    B1 = kmc.dipolar_field(pos, m1, C)
    B2 = kmc.dipolar_field(pos, m2, C)
    B12 = kmc.dipolar_field(pos, 2.0 * m1 - 3.0 * m2, C)
    assert np.allclose(B12, 2.0 * B1 - 3.0 * B2, rtol=1e-12, atol=1e-12 * np.abs(B12).max())
    lhs = math.fsum((m1 * B2).ravel())
    rhs = math.fsum((m2 * B1).ravel())
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1e-300)


def test_two_body_sum_superposes():
    """Field of N particles equals the sum of the N-1 two-body fields (brute force)."""
    rng = np.random.default_rng(5)
    n = 12
    pos = rng.uniform(-60e-9, 60e-9, size=(n, 3))
    m = rng.normal(size=(n, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    B = kmc.dipolar_field(pos, m, _C())
    for i in range(n):
        acc = [[], [], []]
        for j in range(n):
            if j == i:
                continue
            Bij = kmc.dipolar_field(pos[[i, j]], m[[i, j]], _C())[0]
            for c in range(3):
                acc[c].append(Bij[c])
        ref = np.array([math.fsum(a) for a in acc])
        assert np.allclose(B[i], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
