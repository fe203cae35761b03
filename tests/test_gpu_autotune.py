"""Launch-shape autotuner (mh_ctx_autotune / mh_ctx_load_shapes) through the C-ABI.

The tuner times the tiled field kernel's shape candidates and stores the fastest per
bucket; results must stay correct (FP32 field error against the FP64 oracle) and
bitwise reproducible for a given table: alone and in a batch, and on a second context
that loads the saved table."""
import json

import numpy as np
import pytest

from oracle import kmc
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


def _assembly(lib, ctx, n, seed, steps=100):
    R_l = 12e-9 * 0.5 * (n / 0.08) ** (1 / 3)
    pos = W.place_random(n, R_l, 12e-9, seed)
    axes = W.axes_random_3d(n, seed + 1)
    p = lib.Params.make(lib.FP32_FIELD, steps_per_period=steps, n_periods=2, n_discard=1)
    return lib.Assembly(ctx, pos, axes, p), pos, axes, p


def test_autotune_table_and_parity(lib, tmp_path):
    ctx = lib.Context(0)
    path = str(tmp_path / "shapes.json")
    ctx.autotune(lib.FP32_FIELD, [1500, 5000], [1, 3, 12], path)
    table = json.load(open(path))
    print(table)
    keys = {(e["fp64"], e["n_max"], e["groups_max"]) for e in table}
    # 3 replicas share one FP32 group with 1 replica; 12 replicas are 3 groups (bucket 4)
    assert keys == {(0, 2048, 1), (0, 2048, 4), (0, 8192, 1), (0, 8192, 4)}
    for e in table:
        assert e["tile_kind"] in (0, 1) and e["blocks_per_cu"] in (2, 3, 4, 6)
        assert e["us_per_step"] > 0
    # tuned shapes keep the FP32 field within 1e-5 of the FP64 oracle
    a, pos, axes, p = _assembly(lib, ctx, 1500, 61)
    m = np.random.default_rng(3).normal(size=(1500, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    got = a.debug_field(m)
    ref = kmc.dipolar_field(pos, m, kmc.derived(kmc.Params(d=12e-9))["C"])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    a.close()

    # bitwise: alone == batch under the table, and == a context that loads it
    a1, *_ = _assembly(lib, ctx, 1500, 71)
    a2, *_ = _assembly(lib, ctx, 5000, 72)
    a1.run(3, seed=5)
    a1.sync()
    a2.run(12, seed=6)
    a2.sync()
    alone = [a1.replica_areas().copy(), a2.replica_areas().copy(), a2.moments(11).copy()]
    lib.run_batch([a1, a2], [3, 12], [5, 6])
    a1.sync()
    a2.sync()
    assert np.array_equal(a1.replica_areas(), alone[0])
    assert np.array_equal(a2.replica_areas(), alone[1])
    assert np.array_equal(a2.moments(11), alone[2])
    ctx2 = lib.Context(0)
    ctx2.load_shapes(path)
    b2, *_ = _assembly(lib, ctx2, 5000, 72)
    b2.run(12, seed=6)
    b2.sync()
    assert np.array_equal(b2.replica_areas(), alone[1])
    # clearing returns to the built-in rule: same as a fresh context
    ctx.autotune(lib.FP32_FIELD, [])
    ctx3 = lib.Context(0)
    c2, *_ = _assembly(lib, ctx3, 5000, 72)
    a2.run(12, seed=6)
    a2.sync()
    c2.run(12, seed=6)
    c2.sync()
    assert np.array_equal(a2.replica_areas(), c2.replica_areas())
    for x in (a1, a2, b2, c2):
        x.close()


def test_autotune_rejects_bad_input(lib, tmp_path):
    ctx = lib.Context(0)
    for args in ((lib.FP32_FIELD, [1], [1]), (lib.BF16X3_WM, [1000], [1]),
                 (lib.FP32_FIELD, [1000], [0])):
        with pytest.raises(lib.MHError) as e:
            ctx.autotune(*args)
        assert e.value.code == -1
    with pytest.raises(lib.MHError):
        ctx.load_shapes(str(tmp_path / "missing.json"))
    bad = tmp_path / "bad.json"
    bad.write_text('[\n  {"fp64": 0, "n_max": 1000, "groups_max": 1, "tile_kind": 0, '
                   '"blocks_per_cu": 3, "us_per_step": 1.0}\n]\n')   # 1000 is not a bucket
    with pytest.raises(lib.MHError):
        ctx.load_shapes(str(bad))
