"""The latency floor of a resident step (one workgroup exchanging one value per thread
through LDS across one barrier per step, as the step scheme of Sec. II.1 makes each
step depend on the previous one): a positive, finite time per step, below the time per
step of a real resident run (N = 100, FP64, one replica), which does that exchange and
the whole step's arithmetic."""
import time

import numpy as np
import pytest

from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_empty_step_floor_below_resident_step(lib):
    ctx = lib.Context(0)
    floor = ctx.time_empty_steps(6000)
    assert np.isfinite(floor) and floor > 0.0
    a1 = W.lysosome_n100()
    asm = lib.Assembly(ctx, a1.pos, a1.axes, lib.params_from_material(a1.mat, lib.FP64))
    steps = a1.mat.steps_per_period * a1.mat.n_periods
    asm.run(1, seed=a1.seed)
    asm.sync()
    t0 = time.perf_counter()
    asm.run(1, seed=a1.seed)
    asm.sync()
    us_step = (time.perf_counter() - t0) / steps * 1e6
    print(f"empty resident step {floor:.3f} us, N = 100 FP64 step {us_step:.2f} us")
    assert floor < us_step
    with pytest.raises(lib.MHError):
        ctx.time_empty_steps(0)
