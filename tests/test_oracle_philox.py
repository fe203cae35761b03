"""Pins of the oracle's Philox-4x64-10 stream against numpy.random.Philox, an
independent implementation of the same published generator (Salmon et al., SC'11).
The paper only asks for a uniform number per particle and step (Sec. II.1, step vii)."""
import numpy as np

from oracle import philox


def _numpy_block(key, ctr):
    """Block for counter ``ctr`` from numpy: its generator increments the counter
    before producing a block, so the state is set to ctr - 1 (256-bit borrow). Key and
    counter are written into the state directly: the constructor routes large integers
    through a float conversion."""
    v = sum(int(ctr[i]) << (64 * i) for i in range(4))
    v = (v - 1) % (1 << 256)
    c = np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=[0, 0])
    st = bg.state
    st["state"]["counter"] = c
    st["state"]["key"] = np.array([int(key[0]), int(key[1])], dtype=np.uint64)
    st["buffer_pos"] = 4
    bg.state = st
    return bg.random_raw(4)


def test_blocks_match_numpy():
    rng = np.random.default_rng(7)
    cases = [((0, 0), (0, 0, 0, 0)), ((1, 2), (5, 7, 0, 0)),
             ((2**64 - 1, 3), (2**64 - 1, 3, 0, 0)),
             ((123456789, 42), (2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1))]
    for _ in range(20):
        cases.append(((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32))),
                      tuple(int(x) for x in rng.integers(0, 2**63, size=4))))
    for key, ctr in cases:
        ref = _numpy_block(key, ctr)
        got = philox.raw_words(key[0], key[1], np.array([ctr], dtype=np.uint64))[0]
        assert np.array_equal(ref, got), (key, ctr)


def test_uniform_layout():
    seed, stream, k, n = 3001, 5, 1234, 11
    u = philox.uniforms(seed, stream, k, n)
    for i in range(n):
        w = _numpy_block((seed, stream), (i // 4, k, 0, 0))[i % 4]
        assert u[i] == (int(w) >> 11) * 2.0 ** -53
    assert np.all((u >= 0) & (u < 1))


def test_uniform_moments():
    u = philox.uniforms(1, 0, 0, 200000)
    assert abs(u.mean() - 0.5) < 4 * (1 / np.sqrt(12 * 200000))
    assert abs(u.var() - 1 / 12) < 0.002
