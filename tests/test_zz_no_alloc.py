"""mh_field_noalloc, the allocation-free form of mh_debug_field, through the C ABI: on
device buffers, two calls in a row (the second on a smaller assembly) give bitwise the
field mh_debug_field gives for the same moments (same kernels and summation order), the
first call's output survives the second, and both agree with the oracle's Eq. 1 to the
precision's bound. Sizes beyond the fixed scratch array and interaction-matrix
assemblies are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from oracle import kmc
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu

_HIP = None


def hip():
    global _HIP
    if _HIP is None:
        _HIP = C.CDLL("libamdhip64.so")
    return _HIP


def dev_alloc(nbytes):
    p = C.c_void_p()
    assert hip().hipMalloc(C.byref(p), C.c_size_t(nbytes)) == 0
    return p.value


def h2d(dst, arr):
    arr = np.ascontiguousarray(arr, dtype=np.float64)
    assert hip().hipMemcpy(C.c_void_p(dst), arr.ctypes.data_as(C.c_void_p), C.c_size_t(arr.nbytes), 1) == 0


def d2h(src, shape):
    out = np.empty(shape)
    assert hip().hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(src), C.c_size_t(out.nbytes), 2) == 0
    return out


def _unit(n, seed):
    m = np.random.default_rng(seed).normal(size=(n, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def _kw(d):
    return dict(Ms=4e5, Keff=1.3e4, d=d, T=300.0, tau0=1e-10, rho=5200.0, f=1e5, mu0Hmax=0.02,
                steps_per_period=100, n_periods=2, n_discard=1)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def test_noalloc_field_matches_debug_field(ctx, lib):
    # (precision, n, radius, tolerance against the oracle): a tiled FP32 system with
    # source parts, then smaller ones, the last small enough for the resident form
    cases = [(lib.FP32_FIELD, 3000, 180e-9, 1e-5), (lib.FP64, 700, 100e-9, 1e-13),
             (lib.FP64, 100, 80e-9, 1e-13)]
    asms, ms, bufs = [], [], []
    for q, (prec, n, R, _) in enumerate(cases):
        pos = W.place_random(n, R, 12e-9, 1300 + q)
        axes = W.axes_random_3d(n, 1400 + q)
        a = lib.Assembly(ctx, pos, axes, lib.Params.make(prec, **_kw(12e-9)))
        m = _unit(n, 1500 + q)
        dm, dB = dev_alloc(m.nbytes), dev_alloc(m.nbytes)
        h2d(dm, m)
        asms.append((a, pos))
        ms.append(m)
        bufs.append((dm, dB))
    # a finished run on the second assembly: its results must stay as they are
    asms[1][0].run(2, seed=9)
    asms[1][0].sync()
    areas = asms[1][0].replica_areas().copy()
    # calls in a row on the library's stream, each smaller than the one before
    for (a, _), (dm, dB) in zip(asms, bufs):
        a.field_noalloc(dm, dB)
    assert hip().hipDeviceSynchronize() == 0
    got = [d2h(dB, (a.n, 3)) for (a, _), (_, dB) in zip(asms, bufs)]
    for (prec, n, _, tol), (a, pos), m, g in zip(cases, asms, ms, got):
        ref = a.debug_field(m)
        assert np.array_equal(g, ref), np.abs(g - ref).max()
        orc = kmc.dipolar_field(pos, m, kmc.derived(kmc.Params(**_kw(12e-9)))["C"])
        err = np.linalg.norm(g - orc) / np.linalg.norm(orc)
        print(f"precision {prec}, n={n}: bitwise equal to mh_debug_field, oracle error {err:.2e}")
        assert err < tol
    assert np.array_equal(asms[1][0].replica_areas(), areas)
    # a second round on the same buffers, smallest first: the same bits again
    for (a, _), (dm, dB) in reversed(list(zip(asms, bufs))):
        a.field_noalloc(dm, dB)
    assert hip().hipDeviceSynchronize() == 0
    for (a, _), (_, dB), g in zip(asms, bufs, got):
        assert np.array_equal(d2h(dB, (a.n, 3)), g)
    for (a, _), (dm, dB) in zip(asms, bufs):
        hip().hipFree(C.c_void_p(dm))
        hip().hipFree(C.c_void_p(dB))
        a.close()


def test_noalloc_refusals(ctx, lib):
    # an interaction-matrix assembly, and one larger than the fixed array can serve
    n = 64
    pos = W.place_random(n, 60e-9, 12e-9, 1601)
    a = lib.Assembly(ctx, pos, W.axes_random_3d(n, 1602), lib.Params.make(lib.BF16X3_WM, **_kw(12e-9)))
    dm, dB = dev_alloc(n * 24), dev_alloc(n * 24)
    with pytest.raises(lib.MHError) as e:
        a.field_noalloc(dm, dB)
    assert e.value.code == -1
    a.close()
    g = np.arange(60)
    pos = 1.5 * 12e-9 * np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    big = lib.Assembly(ctx, pos, W.axes_random_3d(pos.shape[0], 1603),
                       lib.Params.make(lib.FP64, **_kw(12e-9)))
    dm2, dB2 = dev_alloc(pos.shape[0] * 24), dev_alloc(pos.shape[0] * 24)
    with pytest.raises(lib.MHError) as e:
        big.field_noalloc(dm2, dB2)
    assert e.value.code == -7
    big.close()
    for p in (dm, dB, dm2, dB2):
        hip().hipFree(C.c_void_p(p))
