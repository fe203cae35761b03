"""Batched uneven assemblies (one fused launch sequence for many assemblies of
different sizes, materials, fields and protocols): every assembly's result must be
bitwise the same as when it runs alone with the same replicas and seed, and an FP64
member must still follow the oracle."""
import numpy as np
import pytest

from oracle import kmc
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


def _members(lib):
    rng = np.random.default_rng(31)
    out = []
    specs = [(40, lib.FP64), (150, lib.FP32_FIELD), (300, lib.FP64), (700, lib.FP32_FIELD),
             (1200, lib.FP32_FIELD), (2500, lib.FP32_FIELD), (90, lib.FP32_FIELD),
             (600, lib.BF16X3_WM), (1000, lib.FP64)]
    for q, (n, prec) in enumerate(specs):
        phi = rng.uniform(0.02, 0.15)
        d = rng.uniform(10e-9, 16e-9)
        R = d / 2 * (n / phi) ** (1 / 3)
        pos = W.place_random(n, R, d, 40 + q)
        axes = W.axes_random_3d(n, 60 + q)
        P = int(rng.integers(2, 4))
        kw = dict(Ms=4e5, Keff=float(rng.uniform(0.8e4, 2e4)), d=d, T=300.0, tau0=1e-10,
                  rho=5200.0, f=float(rng.uniform(1e5, 1e6)), mu0Hmax=float(rng.uniform(0.005, 0.04)),
                  steps_per_period=int(rng.choice([60, 100, 140])), n_periods=P, n_discard=1)
        out.append((pos, axes, kw, prec, int(rng.integers(1, 4)), 1000 + q))
    return out


def test_batch_equals_alone(lib):
    ctx = lib.Context(0)
    mem = _members(lib)
    alone = []
    for pos, axes, kw, prec, R, seed in mem:
        a = lib.Assembly(ctx, pos, axes, lib.Params.make(prec, **kw))
        a.run(R, seed)
        a.sync()
        alone.append((a.replica_areas().copy(), [a.moments(r).copy() for r in range(R)],
                      a.loop(0, 0)[1].copy()))
        a.close()
    asms = [lib.Assembly(ctx, pos, axes, lib.Params.make(prec, **kw))
            for pos, axes, kw, prec, R, seed in mem]
    lib.run_batch(asms, [m[4] for m in mem], [m[5] for m in mem])
    for q, a in enumerate(asms):
        a.sync()
        areas = a.replica_areas()
        assert np.array_equal(areas, alone[q][0]), q
        for r in range(mem[q][4]):
            assert np.array_equal(a.moments(r), alone[q][1][r]), (q, r)
        assert np.array_equal(a.loop(0, 0)[1], alone[q][2]), q
    # the FP64 members follow the oracle
    for q, (pos, axes, kw, prec, R, seed) in enumerate(mem):
        if prec != lib.FP64 or len(pos) > 400:
            continue
        ref = kmc.simulate(pos, axes, kmc.Params(**kw), seed=seed, stream=0)
        assert np.abs(asms[q].moments(0) - ref.m_final).max() < 1e-8
        assert abs(asms[q].replica_areas()[0] - ref.area) < 1e-9 * max(1.0, abs(ref.area))
    # a second batch on the same assemblies reuses the captured graph and repeats
    lib.run_batch(asms, [m[4] for m in mem], [m[5] for m in mem])
    for q, a in enumerate(asms):
        a.sync()
        assert np.array_equal(a.replica_areas(), alone[q][0]), q


def test_update_forms_agree_across_the_launch_threshold(lib):
    """A small tiled assembly alone launches the three-role update kernel (few blocks);
    batched with a large one, the launch exceeds 256 blocks and uses the single-role
    kernel. Its results must be bitwise the same either way, in FP32 and FP64."""
    ctx = lib.Context(0)
    kw = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
              mu0Hmax=0.02, steps_per_period=100, n_periods=2, n_discard=1)
    for prec in (lib.FP32_FIELD, lib.FP64):
        pos = W.place_random(1500, 120e-9, 12e-9, 71)
        axes = W.axes_random_3d(1500, 72)
        small = lib.Assembly(ctx, pos, axes, lib.Params.make(prec, **kw))
        small.run(3, seed=5)
        small.sync()
        alone = (small.replica_areas().copy(), small.moments(2).copy(),
                 small.loop(1, 0)[1].copy())
        pos2 = W.place_random(4000, 170e-9, 12e-9, 73)
        big = lib.Assembly(ctx, pos2, W.axes_random_3d(4000, 74),
                           lib.Params.make(lib.FP32_FIELD, **kw))
        lib.run_batch([small, big], [3, 80], [5, 6])   # 3 x 6 + 80 x 16 = 1298 update blocks
        small.sync()
        big.sync()
        assert np.array_equal(small.replica_areas(), alone[0])
        assert np.array_equal(small.moments(2), alone[1])
        assert np.array_equal(small.loop(1, 0)[1], alone[2])
        small.close()
        big.close()


def test_loop_record_slots_agree(lib, tmp_path):
    """An assembly with at most 256 update blocks keeps one loop-record partial sum per
    wave (it may run under the three-role kernel); a larger one keeps one total per
    block. The same replica's loop and area must be bitwise the same either way: one
    replica of a 300-particle FP64 assembly (2 blocks) against the same replica among
    200 (400 blocks), both with 16-target field tiles (a loaded shape table, so that
    the field sums run in the same order)."""
    ctx = lib.Context(0)
    path = tmp_path / "shapes.json"
    path.write_text('[\n'
                    '  {"fp64": 1, "n_max": 512, "groups_max": 1, "tile_kind": 1, '
                    '"blocks_per_cu": 3, "us_per_step": 1.0},\n'
                    '  {"fp64": 1, "n_max": 512, "groups_max": 256, "tile_kind": 1, '
                    '"blocks_per_cu": 3, "us_per_step": 1.0}\n]\n')
    ctx.load_shapes(str(path))
    kw = dict(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
              mu0Hmax=0.02, steps_per_period=100, n_periods=2, n_discard=1)
    pos = W.place_random(300, 60e-9, 12e-9, 81)
    axes = W.axes_random_3d(300, 82)
    a = lib.Assembly(ctx, pos, axes, lib.Params.make(lib.FP64, **kw))
    a.run(1, seed=9)
    a.sync()
    one = (a.replica_areas()[0], a.moments(0).copy(), a.loop(0, 0)[1].copy())
    a.run(200, seed=9)
    a.sync()
    assert a.replica_areas()[0] == one[0]
    assert np.array_equal(a.moments(0), one[1])
    assert np.array_equal(a.loop(0, 0)[1], one[2])
    a.close()
