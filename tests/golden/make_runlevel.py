"""Writes the oracle's per-replica loop areas for the run-level parity tests.

    python tests/golden/make_runlevel.py [case ...]

Each case is one assembly run by ``oracle.kmc.simulate`` for every replica r on the
Philox stream (seed, r), the protocol of Sec. III.1 (loops averaged over runs that
differ in their random numbers and, here, in their easy axes: replica r takes axis set
r, the paper's first averaging method). The area of a replica is the mean over its
particles and kept periods (Sec. III.2.a). Inputs come from the seeded generators of
``paper_1407_2737_amd.workloads``; nothing here calls the GPU library. Replicas run in
a process pool, one thread each.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import kmc  # noqa: E402
from paper_1407_2737_amd import workloads as W  # noqa: E402

# name: (n, lysosome radius, d, placement seed, axes seed, replicas, Philox seed, params)
CASES = {
    "n150_s200": dict(n=150, radius=90e-9, d=12e-9, pos_seed=903, axes_seed=904, R=64,
                      seed=4321, kw=dict(steps_per_period=200, n_periods=2, n_discard=1)),
    "n1400_s100": dict(n=1400, radius=160e-9, d=12e-9, pos_seed=905, axes_seed=906, R=64,
                       seed=2468, kw=dict(steps_per_period=100, n_periods=2, n_discard=1)),
}
BASE = dict(Ms=4e5, Keff=1.3e4, T=300.0, tau0=1e-10, rho=5200.0, f=1e5, mu0Hmax=0.02)


def inputs(c):
    pos = W.place_random(c["n"], c["radius"], c["d"], c["pos_seed"])
    axes = W.axes_random_3d(c["n"] * c["R"], c["axes_seed"]).reshape(c["R"], c["n"], 3)
    p = kmc.Params(**dict(BASE, d=c["d"], **c["kw"]))
    return pos, axes, p


def _one(job):
    name, r = job
    from threadpoolctl import threadpool_limits
    c = CASES[name]
    pos, axes, p = inputs(c)
    with threadpool_limits(1):
        res = kmc.simulate(pos, axes[r], p, seed=c["seed"], stream=r)
    return r, res.area


def path(name):
    return os.path.join(HERE, f"runlevel_{name}.txt")


def main(names):
    import multiprocessing as mp
    for name in names:
        c = CASES[name]
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
            out = dict(pool.map(_one, [(name, r) for r in range(c["R"])]))
        areas = np.array([out[r] for r in range(c["R"])])
        with open(path(name), "w") as f:
            f.write(f"# oracle per-replica loop areas (J/m^3), case {name}: {c}\n")
            f.write(f"# material {BASE}; Sec. III.1 protocol, Sec. III.2.a area\n")
            f.write("# written by tests/golden/make_runlevel.py (oracle only)\n")
            for r, a in enumerate(areas):
                f.write(f"{r} {float(a)!r}\n")
        print(f"{name}: {c['R']} replicas in {time.perf_counter() - t0:.0f} s, mean area "
              f"{areas.mean():.6g} +- {areas.std(ddof=1) / np.sqrt(len(areas)):.3g}", flush=True)


def load(name):
    d = np.loadtxt(path(name))
    return d[:, 1]


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
