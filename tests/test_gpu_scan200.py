"""The paper-literal extremum search (Sec. II.1 step iv taken literally: dE/dtheta on
200 grid angles, each sign change refined by Newton's method) on the GPU against the
oracle's, through the C-ABI:

* the fall for reduced fields (hx, hy) and start angles, including fields just inside
  the astroid where the scan misses the saddle/minimum pair and keeps one well;
* the fused single step (fields, P, jump decisions, new moments) in the resident,
  tiled FP64, tiled FP32 and matrix forms;
* a whole T = 0 loop over random axes, identical to the oracle's;
* rejections: an unknown mode, the mean-magnetisation loop (exact search only)."""
import numpy as np
import pytest

from oracle import kmc, sw
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _params(lib, precision, **kw):
    base = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
                mu0Hmax=0.02, steps_per_period=2000, n_periods=3, n_discard=2,
                extrema_mode=1)
    base.update(kw)
    return lib.Params.make(precision, **base), kmc.Params(**base)


def _rand_moments(n, seed):
    m = np.random.default_rng(seed).normal(size=(n, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def test_fall_scan200_matches_oracle(ctx, lib):
    rng = np.random.default_rng(26)
    n = 20000
    h = rng.uniform(0, 2.0, n) ** 1.5
    phi = rng.uniform(0, np.pi, n)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    hx[:300] = rng.uniform(-1.5, 1.5, 300)
    hy[:300] = 0.0
    hx[300:600] = 0.0
    hy[300:600] = rng.uniform(0, 1.5, 300)
    psi = rng.uniform(0.05, np.pi / 2 - 0.05, 1000)
    hsw = (np.cos(psi) ** (2 / 3) + np.sin(psi) ** (2 / 3)) ** -1.5
    hh = hsw * (1 - 10 ** rng.uniform(-7, -1, 1000))
    hx[600:1600], hy[600:1600] = hh * np.cos(psi), hh * np.sin(psi)
    th0 = rng.uniform(-np.pi, np.pi, n)
    out = ctx.debug_sw(hx, hy, th0, extrema_mode=lib.EXTREMA_SCAN200)
    th, mn, cnt = sw.stationary_points_scan200(hx, hy)
    tc, ec, to, eo, e3, two = sw.classify(th0, th, mn, cnt, hx, hy)
    _, _, cnt_exact = sw.stationary_points(hx, hy)
    missed = (cnt_exact == 4) & (cnt == 2)
    print(f"scan misses the pair in {missed.sum()} of 1000 near-switching fields")
    assert missed[600:1600].sum() > 100
    assert np.array_equal(out[:, 5] == 1.0, two)
    assert np.abs(np.angle(np.exp(1j * (out[:, 0] - tc)))).max() < 1e-12
    assert np.abs(np.angle(np.exp(1j * (out[two, 2] - to[two])))).max() < 1e-12
    assert np.abs(out[:, 1] - ec).max() < 1e-12
    assert np.abs(out[two, 3] - eo[two]).max() < 1e-12
    assert np.abs(out[two, 4] - e3[two]).max() < 1e-12
    # the exact mode of the same entry point is mh_debug_sw
    assert np.array_equal(ctx.debug_sw(hx, hy, th0, extrema_mode=lib.EXTREMA_EXACT),
                          ctx.debug_sw(hx, hy, th0))


# (n, precision, replicas, interactions): 100 particles run resident; 700 FP64 and
# 1500 FP32 run tiled; the matrix form without interactions has the oracle's exact field
@pytest.mark.parametrize("n,prec,nrep,inter", [(100, 0, 2, 1), (700, 0, 2, 1), (1500, 1, 3, 1),
                                               (300, 2, 2, 0)])
def test_single_step_scan200(ctx, lib, n, prec, nrep, inter):
    R_l = 80e-9 * (n / 100) ** (1 / 3)
    pos = W.place_random(n, R_l, 12e-9, 900 + n)
    axes = W.axes_random_3d(n, 901 + n)
    pg, pk = _params(lib, prec, interactions=inter)
    a = lib.Assembly(ctx, pos, axes, pg)
    seed = 777
    m_in = np.stack([_rand_moments(n, 30 + r) for r in range(nrep)])
    for k in (0, 500, 1001, 2999):
        diag = a.debug_steps(nrep, seed, k, k + 1, m_in.reshape(-1, 3))
        for r in range(nrep):
            m_new, info = kmc.step(pos, axes, m_in[r], k, pk, seed, r)
            m_gpu = a.moments(r)
            if prec == 1:
                dif = (diag[r, :, 4] == 1.0) != info.jump
                assert np.all((np.abs(info.u - info.P) < 1e-4)[dif])
                # FP32 fields move (hx, hy) by ~1e-6: a pair count may differ only for
                # the rare field that close to a decision
                assert np.count_nonzero((diag[r, :, 5] == 1.0) != info.two) <= 2
                same = ~dif
                assert np.abs(m_gpu[same] - m_new[same]).max() < 1e-4
            else:
                assert np.array_equal(diag[r, :, 5] == 1.0, info.two)
                assert np.array_equal(diag[r, :, 4] == 1.0, info.jump)
                assert np.abs(diag[r, :, 3] - info.P).max() < 1e-12
                assert np.abs(m_gpu - m_new).max() < 1e-10
    a.close()


def test_T0_loop_scan200_matches_oracle(ctx, lib):
    """A deterministic loop (T = 0, no interactions, 160 particles with stratified random
    axes, 2 periods of 2000 steps): the moments of every kept step equal the oracle's."""
    n = 160
    c = (np.arange(n) + 0.5) / n
    az = np.arange(n) * np.pi * (3 - np.sqrt(5))
    s = np.sqrt(1 - c * c)
    axes = np.stack([c, s * np.cos(az), s * np.sin(az)], axis=1)
    pos = W.place_random(n, 200e-9, 12e-9, 5)
    pg, pk = _params(lib, lib.FP64, T=0.0, mu0Hmax=1.2 * 0.065, n_periods=2, n_discard=1,
                     interactions=0)
    a = lib.Assembly(ctx, pos, axes, pg)
    a.run(1, seed=3)
    a.sync()
    H, M = a.loop(0, 0)
    ref = kmc.simulate(pos, axes, pk, seed=3, stream=0)
    assert np.abs(M - ref.M[0]).max() < 1e-9 * pk.Ms
    assert np.abs(a.moments(0) - ref.m_final).max() < 1e-10
    assert abs(a.sar()["area"] - ref.area) < 1e-9 * abs(ref.area)
    a.close()


def test_scan200_rejections(ctx, lib):
    n = 50
    pos = W.place_random(n, 60e-9, 12e-9, 1)
    axes = W.axes_random_3d(n, 2)
    pg, _ = _params(lib, lib.FP64, extrema_mode=2)
    with pytest.raises(lib.MHError) as e:
        lib.Assembly(ctx, pos, axes, pg)
    assert e.value.code == -1
    pg, _ = _params(lib, lib.FP64, interactions=0)
    a = lib.Assembly(ctx, pos, axes, pg)
    with pytest.raises(lib.MHError) as e:
        a.run_mean_loop(2)
    assert e.value.code == -1
    a.close()
    with pytest.raises(lib.MHError) as e:
        ctx.debug_sw([0.1], [0.2], [0.0], extrema_mode=2)
    assert e.value.code == -1
