"""Philox-4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11), vectorised over counters with numpy uint64 arithmetic.

The paper only says that a random number between 0 and 1 is drawn per particle and
step (Sec. II.1, step vii). The stream used on both sides of the parity check is:

    key     = (seed, stream)                    stream = replica index
    counter = (i // 4, k, 0, 0)                 i = particle index, k = global step
    word    = output word (i mod 4) of that block
    u       = (word >> 11) * 2**-53             53-bit uniform in [0, 1)

Pinned in tests against numpy.random.Philox, which implements the same generator.
"""
import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 128-bit product of two uint64 arrays, returned as (hi, lo)."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(ctr, key, rounds: int = 10):
    """Philox-4x64 bijection. ``ctr``: uint64 array (..., 4); ``key``: uint64 (..., 2)
    broadcastable against ``ctr``. Returns uint64 array (..., 4)."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(ctr[..., i], dtype=np.uint64).copy() for i in range(4))
        k0 = np.asarray(key[..., 0], dtype=np.uint64).copy()
        k1 = np.asarray(key[..., 1], dtype=np.uint64).copy()
        for r in range(rounds):
            if r:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, x0)
            hi1, lo1 = _mulhilo(_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms(seed: int, stream: int, k: int, n: int) -> np.ndarray:
    """The n uniforms in [0,1) drawn at global step ``k`` for particles 0..n-1."""
    nb = (n + 3) // 4
    ctr = np.zeros((nb, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nb, dtype=np.uint64)
    ctr[:, 1] = np.uint64(k)
    key = np.array([seed, stream], dtype=np.uint64)
    words = philox4x64(ctr, key[None, :]).reshape(-1)[:n]
    return (words >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def raw_words(seed: int, stream: int, ctr_rows: np.ndarray) -> np.ndarray:
    """Raw output blocks for explicit counters (rows of 4 uint64)."""
    key = np.array([seed, stream], dtype=np.uint64)
    return philox4x64(np.asarray(ctr_rows, dtype=np.uint64), key[None, :])
