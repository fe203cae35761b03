"""GPU parity of the HIP path against the FP64 oracle, through the C-ABI.

Kernel level (one step from the same snapshot): Philox words bit-exact; Stoner-Wohlfarth
extrema and basin; Eq. 1 fields (FP64 ~1e-12, FP32 <= 1e-5 norm-wise); the whole fused
step (fields, P, jump decisions, new moments). Run level: the FP64 config of 100
particles run for 6000 steps makes the same jump decisions as the oracle."""
import numpy as np
import pytest

from oracle import kmc, philox, sw
from _parity import check_reduced_step
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _params(lib, precision, **kw):
    base = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
                mu0Hmax=0.02, steps_per_period=2000, n_periods=3, n_discard=2)
    base.update(kw)
    return lib.Params.make(precision, **base), kmc.Params(**{k: v for k, v in base.items()})


def _rand_moments(n, seed):
    m = np.random.default_rng(seed).normal(size=(n, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def test_philox_bit_exact(ctx):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**63, size=(5000, 4), dtype=np.int64).astype(np.uint64)
    ctr[:10, 0] = np.uint64(2**64 - 1)
    for seed, stream in ((0, 0), (3001, 7), (2**63 + 5, 2**40)):
        got = ctx.debug_philox(seed, stream, ctr)
        ref = philox.raw_words(seed, stream, ctr)
        assert np.array_equal(got, ref)


def test_sw_extrema_and_fall(ctx):
    rng = np.random.default_rng(2)
    n = 20000
    h = rng.uniform(0, 2.0, n) ** 1.5
    phi = rng.uniform(0, np.pi, n)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    # exact special cases: field along / across the axis, zero field
    hx[:200] = rng.uniform(-1.5, 1.5, 200)
    hy[:200] = 0.0
    hx[200:400] = 0.0
    hy[200:400] = rng.uniform(0, 1.5, 200)
    hx[400:410] = 0.0
    hy[400:410] = 0.0
    th0 = rng.uniform(-np.pi, np.pi, n)
    got = ctx.debug_sw(hx, hy, th0)
    th, mn, cnt = sw.stationary_points(hx, hy)
    tc, ec, to, eo, e3, two = sw.classify(th0, th, mn, cnt, hx, hy)
    assert np.array_equal(got[:, 5] == 1.0, two)
    dc = np.abs(np.angle(np.exp(1j * (got[:, 0] - tc))))
    do = np.abs(np.angle(np.exp(1j * (got[:, 2] - to))))
    assert dc.max() < 1e-11, dc.max()
    assert np.all(do[two] < 1e-11)
    assert np.abs(got[:, 1] - ec).max() < 1e-12
    assert np.abs(got[two, 3] - eo[two]).max() < 1e-12
    assert np.abs(got[two, 4] - e3[two]).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2, 100, 256, 257, 700, 1500])
def test_dipolar_field_fp64(ctx, lib, n):
    R = 40e-9 * max(1.0, (n / 30) ** (1 / 3))
    pos = W.place_random(n, R, 12e-9, 100 + n)
    axes = W.axes_random_3d(n, 200 + n)
    pg, pk = _params(lib, lib.FP64)
    a = lib.Assembly(ctx, pos, axes, pg)
    m = _rand_moments(n, n)
    got = a.debug_field(m)
    ref = kmc.dipolar_field(pos, m, kmc.derived(pk)["C"])
    if n == 1:
        assert np.all(got == 0)
        return
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, err


@pytest.mark.parametrize("n", [100, 257, 3000, 5000])
def test_dipolar_field_fp32(ctx, lib, n):
    R = {100: 80e-9, 257: 90e-9, 3000: 220e-9, 5000: 250e-9}[n]
    pos = W.place_random(n, R, 12e-9, 300 + n)
    axes = W.axes_random_3d(n, 400 + n)
    pg, pk = _params(lib, lib.FP32_FIELD)
    a = lib.Assembly(ctx, pos, axes, pg)
    for seed in (1, 2):
        m = _rand_moments(n, seed)
        got = a.debug_field(m)
        ref = kmc.dipolar_field(pos, m, kmc.derived(pk)["C"])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"n={n} FP32 field rel Frobenius error {err:.3e}")
        assert err < 1e-5, err


@pytest.mark.parametrize("n,prec,nrep", [(100, 0, 2), (300, 0, 2), (2000, 1, 2), (60, 1, 2),
                                         (1500, 1, 3), (700, 1, 4), (333, 1, 5)])
def test_single_step_parity(ctx, lib, n, prec, nrep):
    R_l = 80e-9 * (n / 100) ** (1 / 3)
    pos = W.place_random(n, R_l, 12e-9, 500 + n)
    axes = W.axes_random_3d(n, 600 + n)
    pg, pk = _params(lib, prec)
    a = lib.Assembly(ctx, pos, axes, pg)
    seed = 4242
    m_in = np.stack([_rand_moments(n, 10 + r) for r in range(nrep)])
    for k in (0, 437, 1000, 2999):
        diag = a.debug_steps(nrep, seed, k, k + 1, m_in.reshape(-1, 3))
        for r in range(nrep):
            m_new, info = kmc.step(pos, axes, m_in[r], k, pk, seed, r)
            m_gpu = a.moments(r)
            Bg = diag[r, :, :3]
            errB = np.linalg.norm(Bg - info.B) / np.linalg.norm(info.B)
            assert errB < (1e-13 if prec == 0 else 2e-6), errB
            if prec == 0:
                assert np.array_equal(diag[r, :, 4] == 1.0, info.jump)
                assert np.abs(diag[r, :, 3] - info.P).max() < 1e-12
                assert np.abs(m_gpu - m_new).max() < 1e-10
            else:
                # FP32 fields: the field within its bound, the FP64 rest of the step to
                # rounding given the GPU's own field
                check_reduced_step(pos, axes, m_in[r], k, pk, seed, r, diag[r], m_gpu, 1e-5)


@pytest.mark.parametrize("prec,nrep", [(1, 1), (1, 2), (1, 3), (1, 4), (0, 1)])
def test_single_step_parity_wide_tiles(lib, tmp_path, prec, nrep):
    """The 64-target field tiles (whose chunks are too long to unroll whole, so their
    pair loop runs on a scalar trip counter) for one to four FP32 replicas sharing the
    pair geometry, and in FP64, forced by a loaded shape table: one fused step against
    the oracle at two step indices."""
    n = 1500
    R_l = 80e-9 * (n / 100) ** (1 / 3)
    pos = W.place_random(n, R_l, 12e-9, 900 + n)
    axes = W.axes_random_3d(n, 901 + n)
    path = tmp_path / "wide.json"
    path.write_text('[\n  {"fp64": %d, "n_max": 2048, "groups_max": 1, "tile_kind": 0, '
                    '"blocks_per_cu": 3, "us_per_step": 1.0}\n]\n' % (1 if prec == 0 else 0))
    c = lib.Context(0)
    c.load_shapes(str(path))
    pg, pk = _params(lib, prec)
    a = lib.Assembly(c, pos, axes, pg)
    seed = 777
    m_in = np.stack([_rand_moments(n, 30 + r) for r in range(nrep)])
    for k in (0, 1234):
        diag = a.debug_steps(nrep, seed, k, k + 1, m_in.reshape(-1, 3))
        for r in range(nrep):
            m_new, info = kmc.step(pos, axes, m_in[r], k, pk, seed, r)
            m_gpu = a.moments(r)
            errB = np.linalg.norm(diag[r, :, :3] - info.B) / np.linalg.norm(info.B)
            print(f"prec={prec} R={nrep} k={k} replica {r}: field error {errB:.2e}")
            assert errB < (1e-13 if prec == 0 else 2e-6), errB
            dif = (diag[r, :, 4] == 1.0) != info.jump
            if prec == 0:
                assert not dif.any()
                assert np.abs(m_gpu - m_new).max() < 1e-10
            else:
                check_reduced_step(pos, axes, m_in[r], k, pk, seed, r, diag[r], m_gpu, 1e-5)
    a.close()
    c.close()


def test_trajectory_n100_fp64(ctx, lib):
    """N=100 in an 80 nm lysosome, FP64, 3 periods of 2000 steps, last kept: the same
    trajectory as the oracle."""
    a_in = W.lysosome_n100()
    mat = a_in.mat
    pg = lib.params_from_material(mat, lib.FP64)
    pk = kmc.Params.from_dict(mat.as_dict())
    a = lib.Assembly(ctx, a_in.pos, a_in.axes, pg)
    a.run(1, seed=a_in.seed)
    a.sync()
    res = a.sar()
    H, M = a.loop(0, 0)
    ref = kmc.simulate(a_in.pos, a_in.axes, pk, seed=a_in.seed, stream=0)
    m_gpu = a.moments(0)
    print(f"lysosome_n100: GPU area {res['area']:.9g}, oracle {ref.area:.9g}; jumps {ref.jumps}")
    assert np.abs(m_gpu - ref.m_final).max() < 1e-8
    assert np.abs(M - ref.M[0]).max() < 1e-6 * pk.Ms
    assert np.abs(H - ref.H).max() < 1e-15
    assert abs(res["area"] - ref.area) < 1e-9 * max(abs(ref.area), 1.0)
    assert abs(res["sar"] - ref.sar) < 1e-9 * max(abs(ref.sar), 1.0)
    # per-particle areas (the per-NP analyses of Sec. III)
    a_np = a.area_per_np(0)
    assert np.abs(a_np - ref.area_per_np).max() < 1e-9 * np.abs(ref.area_per_np).max()


def test_per_replica_amplitudes_fp64(ctx, lib):
    """Replicas at different field amplitudes (Sec. III.2.b sweeps): replica r follows
    the oracle run at its amplitude with Philox stream r."""
    n = 60
    pos = W.place_random(n, 70e-9, 12e-9, 71)
    axes = W.axes_random_3d(n, 72)
    amps = [0.01, 0.02, 0.04]
    pg, pk = _params(lib, lib.FP64, steps_per_period=100, n_periods=2, n_discard=1)
    a = lib.Assembly(ctx, pos, axes, pg)
    a.set_replica_fields(amps)
    a.run(3, seed=99)
    a.sync()
    areas = a.replica_areas()
    for r, h in enumerate(amps):
        pk.mu0Hmax = h
        ref = kmc.simulate(pos, axes, pk, seed=99, stream=r)
        assert np.abs(a.moments(r) - ref.m_final).max() < 1e-9
        assert abs(areas[r] - ref.area) < 1e-9 * max(1.0, abs(ref.area))
        a_np = a.area_per_np(r)
        assert np.abs(a_np - ref.area_per_np).max() < 1e-9 * max(1.0, np.abs(ref.area_per_np).max())
        assert abs(a_np.mean() - areas[r]) < 1e-9 * max(1.0, abs(areas[r]))
        H, M = a.loop(r, 0)
        assert np.abs(H - ref.H).max() < 1e-15


def test_invalid_inputs_rejected(ctx, lib):
    pg, _ = _params(lib, lib.FP64)
    pos = np.array([[0, 0, 0], [5e-9, 0, 0]], dtype=float)      # closer than d = 12 nm
    axes = np.array([[1, 0, 0], [0, 1, 0]], dtype=float)
    with pytest.raises(lib.MHError) as e:
        lib.Assembly(ctx, pos, axes, pg)
    assert e.value.code == -2
    with pytest.raises(lib.MHError):
        lib.Assembly(ctx, np.array([[0, 0, 0.0]]), np.array([[0, 0, 0.0]]), pg)  # zero axis
    bad, _ = _params(lib, lib.FP64, steps_per_period=7)
    with pytest.raises(lib.MHError):
        lib.Assembly(ctx, np.array([[0, 0, 0.0]]), np.array([[0, 0, 1.0]]), bad)
    a = lib.Assembly(ctx, np.array([[0, 0, 0.0]]), np.array([[0, 0, 1.0]]), pg)
    with pytest.raises(lib.MHError) as e:
        a.sar()
    assert e.value.code == lib.ENOTREADY
    with pytest.raises(lib.MHError) as e:
        a.area_per_np(0)
    assert e.value.code == lib.ENOTREADY
    a.run(2, seed=1)
    a.sync()
    with pytest.raises(lib.MHError) as e:
        a.area_per_np(2)
    assert e.value.code == -1
