"""Parity at full benchmark size, in the launch configuration the benchmarks time, on
outputs the FP64 oracle computes directly:

* one assembly of N = 5000 (250 nm lysosome, d = 12 nm), FP32 field, three
  replicas at 10, 20 and 40 mT set as per-replica amplitudes. One step from a random
  snapshot at two step indices, every particle of every replica against the oracle.
* N = 4096 at phi = 10 %, 512 replicas with one axis set each, BF16x3 matrix
  form. One step of all 512 replicas from a random snapshot; four sampled replicas
  against the oracle.

Fields are held to the precision's bound (relative Frobenius 1e-5 for FP32, 1e-4 for
BF16x3, whose measured error is about 4e-6). The FP64 rest of the step, fed the GPU's own
field, must give the GPU's switching probabilities (1e-12) and new moments (1e-10); a jump
decision may differ from the exact-field oracle's only where the draw lies between the
two fields' probabilities."""
import numpy as np
import pytest

from oracle import kmc
from _parity import check_reduced_step
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _unit(shape, seed):
    m = np.random.default_rng(seed).normal(size=shape + (3,))
    return m / np.linalg.norm(m, axis=-1, keepdims=True)


def test_n5000_three_amplitudes_full_size_step(ctx, lib):
    w2 = W.lysosome_n5000()
    amps = (0.010, 0.020, 0.040)
    a = lib.Assembly(ctx, w2.pos, w2.axes, lib.params_from_material(w2.mat, lib.FP32_FIELD))
    a.set_replica_fields(list(amps))
    m_in = _unit((len(amps), w2.n), 300)
    for k in (0, 4321):
        diag = a.debug_steps(len(amps), w2.seed, k, k + 1, m_in.reshape(-1, 3))
        for r, h in enumerate(amps):
            pk = kmc.Params.from_dict(dict(w2.mat.as_dict(), mu0Hmax=h))
            err, nd = check_reduced_step(w2.pos, w2.axes, m_in[r], k, pk, w2.seed, r, diag[r],
                                         a.moments(r), 1e-5)
            print(f"N=5000, k={k}, {h * 1e3:g} mT: field error {err:.2e}, {nd} decisions differ")
    a.close()


def test_n4096_512_replicas_full_size_step(ctx, lib):
    R = 512
    a4 = W.replica_batch_n4096(n_axes_sets=R)
    n = a4.n
    a = lib.Assembly(ctx, a4.pos, a4.axes, lib.params_from_material(a4.mat, lib.BF16X3_WM),
                     n_axes_sets=R)
    m_in = _unit((R, n), 400)
    k = 1500
    diag = a.debug_steps(R, a4.seed, k, k + 1, m_in.reshape(-1, 3))
    pk = kmc.Params.from_dict(a4.mat.as_dict())
    for r in (0, 137, 300, 511):
        axes_r = a4.axes[r * n:(r + 1) * n]
        err, nd = check_reduced_step(a4.pos, axes_r, m_in[r], k, pk, a4.seed, r, diag[r],
                                     a.moments(r), 1e-4)
        print(f"N=4096 x 512, replica {r}: field error {err:.2e}, {nd} decisions differ")
    a.close()
