"""Replica statistics of a result (Sec. III.1 averaging, Sec. III.2.a SAR), which every
run-level tolerance and the server's stopping rule rely on: the library's area mean and
standard error equal the oracle's replica_stats (checked against scipy on the CPU) of
the library's own per-replica areas, for a single run, a batch member and one replica;
SAR and its error are the area's times f / rho.

Also: runs of one context on two HIP streams give bitwise the results of the same runs
made one after the other (the context's plan staging is shared by its runs)."""
import ctypes as C

import numpy as np
import pytest

from oracle import kmc
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _kw(**over):
    kw = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
              mu0Hmax=0.02, steps_per_period=100, n_periods=2, n_discard=1)
    kw.update(over)
    return kw


def _check_stats(a, kw):
    res, areas = a.sar(), a.replica_areas()
    mean, se = kmc.replica_stats(areas)
    assert abs(res["area"] - mean) <= 1e-12 * abs(mean)
    assert abs(res["area_se"] - se) <= 1e-12 * se + 1e-300
    conv = kw["f"] / kw["rho"]
    assert abs(res["sar"] - res["area"] * conv) <= 1e-15 * abs(res["sar"])
    assert abs(res["sar_se"] - res["area_se"] * conv) <= 1e-15 * res["sar_se"] + 1e-300
    return res, areas


def test_replica_se_single_batch_and_one_replica(ctx, lib):
    kw = _kw()
    pa = W.place_random(120, 70e-9, 12e-9, 1701)
    pb = W.place_random(600, 110e-9, 12e-9, 1702)
    a = lib.Assembly(ctx, pa, W.axes_random_3d(120 * 7, 1703), lib.Params.make(lib.FP64, **kw),
                     n_axes_sets=7)
    b = lib.Assembly(ctx, pb, W.axes_random_3d(600, 1704),
                     lib.Params.make(lib.FP32_FIELD, **_kw(mu0Hmax=0.03)))
    # a single run of 37 replicas
    a.run(37, seed=5)
    a.sync()
    res, areas = _check_stats(a, kw)
    assert res["area_se"] > 0 and areas.shape == (37,)
    # batch members
    lib.run_batch([a, b], [7, 5], [6, 7])
    a.sync()
    b.sync()
    _check_stats(a, kw)
    _check_stats(b, _kw(mu0Hmax=0.03))
    # one replica: no spread, the mean is that replica's area
    b.run(1, seed=8)
    b.sync()
    res, areas = _check_stats(b, _kw(mu0Hmax=0.03))
    assert res["area_se"] == 0.0 and res["sar_se"] == 0.0 and res["area"] == areas[0]
    a.close()
    b.close()


def _stream():
    hip = C.CDLL("libamdhip64.so")
    s = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(s)) == 0
    return hip, s


def test_two_streams_match_sequential_runs(ctx, lib):
    kw = _kw(steps_per_period=200)   # 400 steps: graph-replayed
    pa = W.place_random(1500, 140e-9, 12e-9, 1711)
    pb = W.place_random(500, 100e-9, 12e-9, 1712)
    a = lib.Assembly(ctx, pa, W.axes_random_3d(1500, 1713), lib.Params.make(lib.FP32_FIELD, **kw))
    b = lib.Assembly(ctx, pb, W.axes_random_3d(500, 1714), lib.Params.make(lib.FP64, **kw))
    ref = {}
    for name, x, R, seed in (("a", a, 3, 11), ("b", b, 2, 12)):
        x.run(R, seed=seed)
        x.sync()
        ref[name] = (x.replica_areas().copy(), x.moments(R - 1).copy())
    hip, s1 = _stream()
    _, s2 = _stream()
    for _ in range(2):
        a.run(3, seed=11, stream=s1.value)
        b.run(2, seed=12, stream=s2.value)
        a.sync()
        b.sync()
        for name, x, R in (("a", a, 3), ("b", b, 2)):
            assert np.array_equal(x.replica_areas(), ref[name][0])
            assert np.array_equal(x.moments(R - 1), ref[name][1])
    assert hip.hipStreamSynchronize(s1) == 0 and hip.hipStreamSynchronize(s2) == 0
    hip.hipStreamDestroy(s1)
    hip.hipStreamDestroy(s2)
    a.close()
    b.close()
