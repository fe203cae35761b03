"""Per-particle geometry analyses of the paper (test infrastructure, like the rest of
this package).

Local volume concentration, Eq. 8 (Sec. III.5): phi_N = 3 N V / (4 pi r_N^3) with
r_N the distance from the particle to its N-th nearest neighbour and V = pi d^3 / 6
the particle volume, i.e. phi_N = N d^3 / (8 r_N^3).
"""
import numpy as np


def local_concentration(pos: np.ndarray, d: float, N: int) -> np.ndarray:
    """phi_N of every particle (Eq. 8). Squared distances are formed as
    dx*dx + dy*dy + dz*dz; the N-th smallest over the other particles gives r_N."""
    n = pos.shape[0]
    if not 1 <= N <= n - 1:
        raise ValueError("N must lie in [1, n-1]")
    out = np.empty(n)
    for i in range(n):
        q = pos - pos[i]
        d2 = q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2]
        d2 = np.delete(d2, i)
        rN = np.sqrt(np.partition(d2, N - 1)[N - 1])
        out[i] = 3.0 * N * (np.pi * d ** 3 / 6.0) / (4.0 * np.pi * rN ** 3)
    return out
