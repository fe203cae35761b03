"""The paper's own validation (Sec. II.3, Fig. 1(c)-(d)) at its stated settings, on
the GPU: with interactions off, kMC loops averaged over runs superimpose on the
deterministic mean-magnetisation loop (whose kernel matches the FP64 oracle to
rounding, see test_gpu_master.py).

* Fig. 1(c), superparamagnetic regime: K = 1e4 J/m^3, d = 20 nm, mu0 Hmax = 1 mT,
  6000-step loops run 10 times, on 2000 particles with axes random in space (3D) and
  on 4000 with axes random in a plane containing the field (2D).
* Fig. 1(d), ferromagnetic regime: K = 1e6 J/m^3, d = 12 nm, mu0 Hmax = 2.5 T,
  10000-step loops on 400 particles with axes random in space, T = 5, 520, 2000 K.
Other values are the paper's defaults (T = 300 K, M_S = 1e6 A/m, f = 100 kHz,
nu0 = 1e10 Hz); two periods with the first discarded. The kMC runs are 64 replicas
with independent Philox streams (the paper averaged 10 runs; more replicas sharpen the
test). Criteria: area within 4 standard errors over replicas, every loop point within
5.5. In the blocked regime (5 K) switching is a rare event: where no replica jumps the
sample error is 0 while the expected weight is not, so the error has a floor of
sqrt(3) 2 M_S / (n R), the rule-of-three bound on an unobserved count (one jump moves
the replica mean by 2 M_S / (n R)). The runs are seeded, so the outcome is
deterministic."""
import numpy as np
import pytest

from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


CASES = {
    "1c-3D": dict(n=2000, axes="3d", Keff=1e4, d=20e-9, mu0Hmax=1e-3, T=300.0, S=6000, R=64),
    "1c-2D": dict(n=4000, axes="2d", Keff=1e4, d=20e-9, mu0Hmax=1e-3, T=300.0, S=6000, R=64),
    "1d-5K": dict(n=400, axes="3d", Keff=1e6, d=12e-9, mu0Hmax=2.5, T=5.0, S=10000, R=64),
    "1d-520K": dict(n=400, axes="3d", Keff=1e6, d=12e-9, mu0Hmax=2.5, T=520.0, S=10000, R=64),
    "1d-2000K": dict(n=400, axes="3d", Keff=1e6, d=12e-9, mu0Hmax=2.5, T=2000.0, S=10000,
                     R=64),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fig1_kmc_superimposes_on_mean_loop(ctx, lib, name):
    c = CASES[name]
    n, R = c["n"], c["R"]
    axes = (W.axes_random_3d if c["axes"] == "3d" else W.axes_random_2d)(n, 1100 + n)
    # positions do not enter with interactions off; they only have to be valid
    pos = W.place_lattice_disorder(n, 0.5 * c["d"] * (n / 0.01) ** (1 / 3), c["d"], 1200 + n)
    kw = dict(Ms=1e6, Keff=c["Keff"], d=c["d"], T=c["T"], tau0=1e-10, rho=5200.0, f=1e5,
              mu0Hmax=c["mu0Hmax"], steps_per_period=c["S"], n_periods=2, n_discard=1,
              interactions=0)
    a = lib.Assembly(ctx, pos, axes, lib.Params.make(lib.FP32_FIELD, **kw))
    a.run(R, seed=31)
    a.sync()
    res = a.sar()
    Mk = np.array([a.loop(r, 0)[1] for r in range(R)])
    b = lib.Assembly(ctx, pos, axes, lib.Params.make(lib.FP64, **kw))
    b.run_mean_loop(1)
    b.sync()
    A_det = b.replica_areas()[0]
    _, M_det = b.loop(0, 0)
    se_M = Mk.std(axis=0, ddof=1) / np.sqrt(R)
    floor = np.sqrt(3.0) * 2.0 * kw["Ms"] / (n * R)
    z = np.abs(Mk.mean(axis=0) - M_det) / np.maximum(se_M, floor)
    print(f"{name}: kMC area {res['area']:.5g} +- {res['area_se']:.2g} J/m^3, mean loop "
          f"{A_det:.5g}; loop amplitude {np.abs(M_det).max() / kw['Ms']:.3f} M_S; "
          f"max loop z {z.max():.2f}")
    assert abs(res["area"] - A_det) < 4 * res["area_se"] + 1e-6 * abs(A_det) + 1e-9
    assert z.max() < 5.5
    a.close()
    b.close()
