"""The applied field along a chosen direction e_H (field_dir) on the GPU against the
oracle, through the C-ABI: the fused single step (resident and tiled), a whole FP64
trajectory with its loop, per-particle areas and Eq. 6 values, and the deterministic
mean loop; (0, 0, 0) is +x bit for bit; a non-finite direction is rejected."""
import numpy as np
import pytest

from oracle import kmc, master
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu

TILT = (1.0, 2.0, -2.0)          # e_H = (1, 2, -2) / 3


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _params(lib, precision, **kw):
    base = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
                mu0Hmax=0.02, steps_per_period=2000, n_periods=3, n_discard=2, field_dir=TILT)
    base.update(kw)
    return lib.Params.make(precision, **base), kmc.Params(**base)


def _rand_moments(n, seed):
    m = np.random.default_rng(seed).normal(size=(n, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


@pytest.mark.parametrize("n", [120, 900])     # resident, tiled
def test_single_step_tilted_field(ctx, lib, n):
    pos = W.place_random(n, 80e-9 * (n / 100) ** (1 / 3), 12e-9, 40 + n)
    axes = W.axes_random_3d(n, 41 + n)
    pg, pk = _params(lib, lib.FP64)
    a = lib.Assembly(ctx, pos, axes, pg)
    m_in = np.stack([_rand_moments(n, 50 + r) for r in range(2)])
    for k in (0, 333, 1000):
        diag = a.debug_steps(2, 99, k, k + 1, m_in.reshape(-1, 3))
        for r in range(2):
            m_new, info = kmc.step(pos, axes, m_in[r], k, pk, 99, r)
            assert np.linalg.norm(diag[r, :, :3] - info.B) < 1e-13 * np.linalg.norm(info.B)
            assert np.array_equal(diag[r, :, 4] == 1.0, info.jump)
            assert np.abs(diag[r, :, 3] - info.P).max() < 1e-12
            assert np.abs(a.moments(r) - m_new).max() < 1e-10
    a.close()


def test_trajectory_tilted_field_fp64(ctx, lib):
    n = 150
    pos = W.place_random(n, 75e-9, 12e-9, 61)
    axes = W.axes_random_3d(n, 62)
    pg, pk = _params(lib, lib.FP64, steps_per_period=400, n_periods=3, n_discard=1,
                     mu0Hmax=0.03)
    a = lib.Assembly(ctx, pos, axes, pg)
    a.run(1, seed=17)
    a.sync()
    ref = kmc.simulate(pos, axes, pk, seed=17, stream=0)
    assert ref.jumps > 0
    assert np.abs(a.moments(0) - ref.m_final).max() < 1e-8
    for per in range(2):
        H, M = a.loop(0, per)
        assert np.abs(M - ref.M[per]).max() < 1e-6 * pk.Ms
    assert abs(a.sar()["area"] - ref.area) < 1e-9 * max(abs(ref.area), 1.0)
    a_np = a.area_per_np(0)
    assert np.abs(a_np - ref.area_per_np).max() < 1e-9 * np.abs(ref.area_per_np).max()
    dh = a.dhdip(0)
    assert np.abs(dh - ref.dhdip_per_np).max() < 1e-9 * np.abs(ref.dhdip_per_np).max()
    a.close()


def test_mean_loop_tilted_field(ctx, lib):
    n = 200
    axes = W.axes_random_3d(n, 71)
    pos = W.place_random(n, 150e-9, 12e-9, 72)
    pg, pk = _params(lib, lib.FP64, steps_per_period=200, n_periods=2, n_discard=1,
                     interactions=0, mu0Hmax=0.03)
    a = lib.Assembly(ctx, pos, axes, pg)
    a.run_mean_loop(1)
    a.sync()
    H, M = a.loop(0, 0)
    Hr, Mr, Ar = master.mean_loop(axes, pk)
    assert np.abs(M - Mr[0]).max() < 1e-9 * pk.Ms
    assert abs(a.sar()["area"] - Ar) < 1e-9 * abs(Ar)
    a.close()


def test_zero_direction_is_x_and_nonfinite_rejected(ctx, lib):
    n = 300
    pos = W.place_random(n, 90e-9, 12e-9, 81)
    axes = W.axes_random_3d(n, 82)
    out = []
    for fd in ((1.0, 0.0, 0.0), (0.0, 0.0, 0.0)):
        pg, _ = _params(lib, lib.FP32_FIELD, steps_per_period=200, n_periods=2, n_discard=1,
                        field_dir=fd)
        a = lib.Assembly(ctx, pos, axes, pg)
        a.run(2, seed=5)
        a.sync()
        out.append((a.replica_areas().copy(), a.moments(1).copy(), a.loop(1, 0)[1].copy()))
        a.close()
    for x, y in zip(*out):
        assert np.array_equal(x, y)
    pg, _ = _params(lib, lib.FP64, field_dir=(np.nan, 0.0, 1.0))
    with pytest.raises(lib.MHError) as e:
        lib.Assembly(ctx, pos, axes, pg)
    assert e.value.code == -1
