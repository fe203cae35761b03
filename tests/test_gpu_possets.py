"""Position sets (the paper's second averaging method, Sec. III.1): replica r runs with
position set r mod P and axis set r mod A. Each replica must follow the oracle run on its
own geometry; FP32 replicas that share a set are grouped in the field kernel."""
import numpy as np
import pytest

from oracle import kmc
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu
D = 12e-9


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _sets(n, P, radius, seed):
    # lattice + maximal disorder: particle i sits near the same node in every set
    return [W.place_lattice_disorder(n, radius, D, seed + q) for q in range(P)]


def test_fp64_replicas_follow_their_geometry(ctx, lib):
    n, P, A, R = 60, 2, 3, 4
    pos = _sets(n, P, 75e-9, 11)
    axes = [W.axes_random_3d(n, 20 + q) for q in range(A)]
    kw = dict(steps_per_period=100, n_periods=2, n_discard=1)
    a = lib.Assembly(ctx, np.concatenate(pos), np.concatenate(axes),
                     lib.Params.make(lib.FP64, **kw), n_axes_sets=A, n_pos_sets=P)
    a.run(R, seed=5)
    a.sync()
    areas = a.replica_areas()
    for r in range(R):
        ref = kmc.simulate(pos[r % P], axes[r % A], kmc.Params(**kw), seed=5, stream=r)
        assert np.abs(a.moments(r) - ref.m_final).max() < 1e-9
        assert abs(areas[r] - ref.area) < 1e-9 * max(1.0, abs(ref.area))
        assert np.abs(a.dhdip(r) - ref.dhdip_per_np).max() < 1e-9 * np.abs(ref.dhdip_per_np).max()
    a.close()


def test_fp32_grouped_by_set_single_step(ctx, lib):
    n, P, R = 700, 2, 6          # sets {0,2,4} and {1,3,5}: two groups of three
    pos = _sets(n, P, 110e-9, 31)
    axes = W.axes_random_3d(n, 41)
    kw = dict(steps_per_period=2000, n_periods=3, n_discard=2)
    a = lib.Assembly(ctx, np.concatenate(pos), axes, lib.Params.make(lib.FP32_FIELD, **kw),
                     n_pos_sets=P)
    rng = np.random.default_rng(3)
    m_in = rng.normal(size=(R, n, 3))
    m_in /= np.linalg.norm(m_in, axis=2, keepdims=True)
    k = 123
    diag = a.debug_steps(R, 77, k, k + 1, m_in.reshape(-1, 3))
    pk = kmc.Params(**kw)
    for r in range(R):
        m_new, info = kmc.step(pos[r % P], axes, m_in[r], k, pk, 77, r)
        Bg = diag[r, :, :3]
        assert np.linalg.norm(Bg - info.B) / np.linalg.norm(info.B) < 2e-6
        dif = (diag[r, :, 4] == 1.0) != info.jump
        assert np.all(np.abs(info.u - info.P)[dif] < 1e-4)
    a.close()


def test_sets_rejected_where_unsupported(ctx, lib):
    n = 50
    pos = _sets(n, 2, 70e-9, 51)
    axes = W.axes_random_3d(n, 52)
    with pytest.raises(lib.MHError) as e:
        lib.Assembly(ctx, np.concatenate(pos), axes, lib.Params.make(lib.BF16X3_WM), n_pos_sets=2)
    assert e.value.code == -1
    bad = pos[1].copy()
    bad[1] = bad[0] + [0.5 * D, 0, 0]          # overlap in the second set
    with pytest.raises(lib.MHError) as e:
        lib.Assembly(ctx, np.concatenate([pos[0], bad]), axes, lib.Params.make(lib.FP64),
                     n_pos_sets=2)
    assert e.value.code == -2
