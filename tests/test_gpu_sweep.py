"""Concentration dependence of the loop area of large particles (T = 0, the paper's
d -> infinity case, Sec. III.2-3) on the GPU. Dilute assemblies (mu0 Ms^2 phi / K =
0.01, below the 0.02 the paper gives for negligible interactions) must reproduce the
Stoner-Wohlfarth random-axis area from the oracle's independent quadrature; dense ones
(mu0 Ms^2 phi / K = 10) lose area, as the paper reports for fields near the coercive
field. The field is sampled 4000 times per period: switching happens at the first
sample past the switching field, which biases the area up by about 0.6 % here (1.2 % at
2000 steps)."""
import numpy as np
import pytest

from oracle import swloop
from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_dilute_matches_sw_and_dense_loses_area(lib):
    ctx = lib.Context(0)
    n, sets, d, Ms, K, Hmax = 2000, 8, 20e-9, 1e6, 1.3e4, 0.04
    res = {}
    asms = []
    for q, phi in enumerate((1e-4, 0.1)):
        radius = 0.5 * d * (n / phi) ** (1 / 3)
        pos = W.place_lattice_disorder(n, radius, d, 500 + q)
        axes = np.concatenate([W.axes_random_3d(n, 600 + 10 * q + s) for s in range(sets)])
        p = lib.Params.make(lib.FP32_FIELD, Ms=Ms, Keff=K, d=d, T=0.0, mu0Hmax=Hmax,
                            steps_per_period=4000, n_periods=2, n_discard=1)
        asms.append(lib.Assembly(ctx, pos, axes, p, n_axes_sets=sets))
    lib.run_batch(asms, [sets, sets], [1, 2])
    for q, a in enumerate(asms):
        a.sync()
        res[q] = a.sar()
        a.close()
    hk = 2 * K / Ms
    ref = swloop.random_axis_area_over_K(Hmax / hk)
    dilute, dense = res[0]["area"] / K, res[1]["area"] / K
    print(f"A/K dilute {dilute:.4f} +- {res[0]['area_se'] / K:.4f} (SW {ref:.4f}), "
          f"dense {dense:.4f}")
    assert abs(dilute - ref) < max(0.025 * ref, 3 * res[0]["area_se"] / K)
    assert dense < 0.8 * dilute
