"""Eq. 8 local concentration in the oracle, pinned by the neighbour shells of a simple
cubic lattice: an interior node has 6 neighbours at a, 12 at a sqrt 2, 8 at a sqrt 3
and 6 at 2a, so phi_N = N d^3 / (8 r^3) with r the shell radius that holds the N-th."""
import numpy as np
import pytest

from oracle import analysis

D = 12e-9


def _lattice(a, m=3):
    g = np.arange(-m, m + 1) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


@pytest.mark.parametrize("N,shell", [(1, 1.0), (6, 1.0), (7, 2 ** 0.5), (18, 2 ** 0.5),
                                     (19, 3 ** 0.5), (26, 3 ** 0.5), (27, 2.0)])
def test_cubic_lattice_centre(N, shell):
    a = 1.5 * D
    pos = _lattice(a)
    centre = np.argmin(np.linalg.norm(pos, axis=1))
    phi = analysis.local_concentration(pos, D, N)[centre]
    assert phi == pytest.approx(N * D ** 3 / (8 * (shell * a) ** 3), rel=1e-13)


def test_scaling_and_bounds():
    rng = np.random.default_rng(4)
    pos = rng.uniform(-1e-7, 1e-7, size=(40, 3))
    p1 = analysis.local_concentration(pos, D, 5)
    p2 = analysis.local_concentration(2.0 * pos, D, 5)    # lengths x2 -> phi / 8
    assert np.allclose(p2, p1 / 8, rtol=1e-13)
    with pytest.raises(ValueError):
        analysis.local_concentration(pos, D, 40)
