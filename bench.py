"""Throughput of the kMC hysteresis hot path on one MI355X, in NP.steps/s.

Workload (default, the paper-scale plain form): one lysosome of radius 250 nm holding
5000 hard spheres of 12 nm (phi = 6.9 %), random 3-D easy axes, Ms = 4e5 A/m,
K = 1.3e4 J/m^3, T = 300 K, tau0 = 1e-10 s, 100 kHz, at three field amplitudes
(10, 20, 40 mT) run together as three replicas of the assembly (one per amplitude, on
their own Philox streams), 5 periods of 2000 steps (first discarded). Dipolar sum in
FP32, per-particle barrier step and area in FP64.

One bench step = one complete run of the batch (all 3 x 5 x 2000 time steps, each with
every part of the path: dipolar field, Stoner-Wohlfarth extrema, switching draw, area
accumulation, then the SAR reduction). value = NP.steps executed / wall time, with the
inputs already resident in device memory.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-secondary]

Prints one JSON line. Its roofline entry is for the dominant kernel (the tiled field
sum): algorithmic flops per launch (29 per pair and replica, Eq. 1) over the kernel's
mean duration, which mh_time_kernels measures with HIP events on graph replays of the
timed run's own plan. Unless --no-secondary, the line also carries "secondary" lines for
the other single-GPU configurations, each timed in the same process: N=100 in FP64 (one
resident launch per run), 256 uneven assemblies with autotuned shapes, and 512 replicas
of N=4096 in the interaction-matrix form on MFMA.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak, FLOP/s
PEAK_FP64_VECTOR = 78.6e12      # MI355X published FP64 vector peak, FLOP/s
PEAK_BF16_MFMA = 2.5e15         # MI355X dense BF16 matrix peak, FLOP/s
FLOPS_PER_PAIR = 29             # Eq. 1 pair term per system (FMA = 2): 3 differences, 5 for
                                # r^2, 2 for r^-3, 5 for m.r, 2 for the 3 (m.r)/r^2 factor,
                                # 12 for the accumulation; the reciprocal square root aside
GEOM_FLOPS = 12                 # executed: pair geometry once per replica group
MOMENT_FLOPS = 18               # executed: moment part per replica
ALG_BYTES_PER_NP = 48           # HBM bytes per particle and system per step of the plain
                                # form: position, moment in, field out (16 B each)

# HBM bytes per launch of the dominant kernel, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE over the default workload, each scaled by what the counter reads for a
# 256 MiB elementwise copy (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000); tied to the kernel
# as measured (profiles/k_field_n5000x3_fp32.md). None where no such measurement exists.
TRAFFIC_BYTES = {"k_field<float,16,3>": (1412.69 * 2.000 + 703.13 * 1.000) * 1024}


_POOL_ASM = None  # the workload the pooled oracle leg steps (set before the fork)


def _oracle_replica_steps(job):
    """One worker of the pooled oracle leg: steps of replica r for budget_s seconds."""
    r, budget_s = job
    from threadpoolctl import threadpool_limits
    from oracle import kmc
    a = _POOL_ASM
    with threadpool_limits(1):
        p = kmc.Params.from_dict(a.mat.as_dict())
        m = kmc.initial_moments(a.axes)
        t0 = time.perf_counter()
        k = 0
        while k < 200 and time.perf_counter() - t0 < budget_s:
            m, _ = kmc.step(a.pos, a.axes, m, k, p, a.seed, r)
            k += 1
    return k


def cpu_baseline(assemblies, budget_s=15.0, pool_s=10.0):
    """The FP64 oracle on the host, on a bounded number of steps of the same workload:
    single-threaded, then one process per core (at most 16) over replicas. Runs before
    the GPU is touched, so that the pool's processes fork from a host-only process."""
    global _POOL_ASM
    import multiprocessing as mp
    import os
    from threadpoolctl import threadpool_limits
    from oracle import kmc
    a = assemblies[1]
    p = kmc.Params.from_dict(a.mat.as_dict())
    m = kmc.initial_moments(a.axes)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        k = 0
        while True:
            m, _ = kmc.step(a.pos, a.axes, m, k, p, a.seed, 0)
            k += 1
            if time.perf_counter() - t0 > budget_s or k >= 200:
                break
        dt = time.perf_counter() - t0
    procs = max(1, min(16, os.cpu_count() or 1))
    _POOL_ASM = a
    with mp.get_context("fork").Pool(procs) as pool:
        t1 = time.perf_counter()
        ks = pool.map(_oracle_replica_steps, [(r, pool_s) for r in range(procs)])
        dt_pool = time.perf_counter() - t1
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         None)
    except OSError:
        pass
    return {"value": a.n * k / dt, "unit": "NP·steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} steps of the 20 mT assembly (N={a.n}), single-threaded numpy FP64",
            "host": {"cpu_model": model, "os_cpu_count": os.cpu_count()},
            "pool": {"value": a.n * sum(ks) / dt_pool, "cores": procs,
                     "sample": f"{procs} processes, one replica each (own Philox stream), "
                               f"{sum(ks)} steps in all of the same assembly, one thread each"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--periods", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="default workload only: skip the secondary lines (N=100, 256 uneven "
                         "assemblies, 512-replica matrix form)")
    ap.add_argument("--no-tune", action="store_true", help="uneven256: built-in launch-shape rule")
    ap.add_argument("--workload", default="n5000",
                    choices=["n100", "n5000", "uneven256", "replicas512", "replicas512plain",
                             "served", "master", "sweep", "methods", "figs"])
    ap.add_argument("--requests", type=int, default=24, help="served: requests per arrival rate")
    ap.add_argument("--sat-requests", type=int, default=8, help="served: saturation requests")
    ap.add_argument("--rates", default="0.5,0.7,0.9", help="served: factors of the plain "
                    "engine's saturated request rate")
    ap.add_argument("--max-replicas", type=int, default=512)
    ap.add_argument("--engines", default="plain,matrix", help="served: plain and/or matrix")
    ap.add_argument("--lambda0", type=float, default=0.0,
                    help="served: the plain engine's saturated request rate (req/s) when it "
                         "is not measured in this run")
    ap.add_argument("--assemblies", type=int, default=256)
    ap.add_argument("--replicas", type=int, default=512)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path is a single-device build; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import paper_1407_2737_amd as mh
    from paper_1407_2737_amd import workloads as W

    single = {"uneven256": bench_uneven256, "master": bench_master, "n100": bench_n100,
              "sweep": bench_sweep, "methods": bench_methods, "figs": bench_figs,
              "served": bench_served,
              "replicas512": bench_replicas512, "replicas512plain": bench_replicas512}
    if args.workload in single:
        line = single[args.workload](args, mh, W)
        if line is not None:
            print(json.dumps(line), flush=True)
        return
    line = bench_n5000(args, mh, W)
    if not args.no_secondary:
        # the other single-GPU benchmark configurations, each timed here on its own:
        # a few complete runs after one warm-up run, kernel durations on the same plan
        sec = argparse.Namespace(**vars(args))
        sec.steps, sec.warmup, sec.periods = 2, 1, 3
        line["secondary"] = [bench_n100(sec, mh, W), bench_uneven256(sec, mh, W),
                             bench_replicas512(argparse.Namespace(**dict(vars(sec),
                                               workload="replicas512")), mh, W)]
    print(json.dumps(line), flush=True)


def _roof(bound, alg, us, peak, unit, kernel, **extra):
    """Roofline entry of one kernel: algorithmic work per launch over its duration."""
    ach = alg / (us * 1e-6)
    out = {"bound": bound, "achieved": ach / 1e12, "peak": peak / 1e12, "unit": unit,
           "frac": ach / peak, "kernel": kernel, "avg_launch_us": us,
           "work_per_launch": alg}
    out.update(extra)
    return out


def bench_n5000(args, mh, W):
    """The default workload: one 5000-particle lysosome at three amplitudes."""
    import numpy as np
    amps = (0.010, 0.020, 0.040)
    w2 = W.lysosome_n5000(n_periods=args.periods)
    work = [w2] * len(amps)
    cpu = None if args.no_cpu else cpu_baseline(work)
    ctx = mh.Context(0)
    # one lysosome, one replica per amplitude (Philox stream = replica index)
    asm = mh.Assembly(ctx, w2.pos, w2.axes, mh.params_from_material(w2.mat, mh.FP32_FIELD))
    asm.set_replica_fields(amps)
    n_total = w2.n * len(amps)
    steps_per_run = w2.mat.steps_per_period * w2.mat.n_periods

    def one_run():
        asm.run(len(amps), seed=w2.seed)
        asm.sync()
        ar = asm.replica_areas()
        return [{"sar": x * w2.mat.f / w2.mat.rho} for x in ar]

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_run()
    t1 = time.perf_counter()
    wall = t1 - t0
    np_steps = n_total * steps_per_run * args.steps
    value = np_steps / wall
    us_step = wall / (args.steps * steps_per_run) * 1e6
    # per-particle area against depth below the membrane, 1 - |r|/R (the output of this
    # workload): mean per-particle area of each amplitude in depth bins of the last run
    depth = 1.0 - np.linalg.norm(w2.pos, axis=1) / w2.radius
    edges = [0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 1.0]
    which = np.digitize(depth, edges[1:-1])
    profile, dh_profile, corr = {}, {}, {}
    for r, h in enumerate(amps):
        a_np = asm.area_per_np(r)
        dh = asm.dhdip(r)                     # Eq. 6 per particle
        key = f"{h * 1e3:g} mT"
        profile[key] = [float(a_np[which == b].mean()) for b in range(len(edges) - 1)]
        dh_profile[key] = [float(dh[which == b].mean() * 1e3) for b in range(len(edges) - 1)]
        corr[key] = float(np.corrcoef(dh, a_np)[0, 1])
    phi20 = asm.local_concentration(20)      # Eq. 8
    field_err = {f"{h * 1e3:g} mT": asm.field_error(r)[0] for r, h in enumerate(amps)}
    analyses = {"dhdip_mT_vs_depth": dh_profile, "corr_dhdip_area": corr,
                "phi20_vs_depth": [float(phi20[which == b].mean()) for b in range(len(edges) - 1)]}
    # kernel durations on the timed run's plan: 50 steps of launches of one kind,
    # replayed back to back from a graph (the update replay overwrites the run's state,
    # so it comes after every result above has been read)
    us_field = mh.time_kernels([asm], 0, 50, 40)
    us_update = mh.time_kernels([asm], 3, 50, 40)
    pairs = sum(w.n * (w.n - 1) for w in work)
    alg_bytes = ALG_BYTES_PER_NP * n_total
    traffic = TRAFFIC_BYTES.get("k_field<float,16,3>")
    roofline = _roof("alu", FLOPS_PER_PAIR * pairs, us_field, PEAK_FP32_VECTOR, "TFLOP/s",
                     "k_field<float,16,3>", traffic=traffic,
                     traffic_over_algorithmic=traffic / alg_bytes if traffic else None,
                     algorithmic_bytes_per_launch=alg_bytes,
                     executed_flops_per_launch=GEOM_FLOPS * w2.n * (w2.n - 1) + MOMENT_FLOPS * pairs,
                     update_us_per_step=us_update,
                     kernels_over_step=(us_field + us_update) / us_step,
                     timing="graph replay of 50 steps x 40 on the timed run's plan, HIP events")
    line = {
        "metric": "NP·steps/s (dipolar+kMC)",
        "value": value,
        "unit": "NP·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 field / f64 barrier",
        "data": "synthetic",
        "config": {"workload": "N=5000 in a 250 nm lysosome, d=12 nm (phi=6.9%), "
                               "random 3-D axes, 10/20/40 mT batched, 100 kHz, "
                               f"{args.periods} periods x 2000 steps",
                   "n_particles_total": n_total, "steps_per_run": steps_per_run,
                   "us_per_time_step": us_step,
                   "sar_W_per_g": [r["sar"] / 1e3 for r in res],
                   "area_Jm3_vs_depth": {"depth_edges": edges,
                                         "count": [int((which == b).sum())
                                                   for b in range(len(edges) - 1)],
                                         **profile},
                   "per_particle_analyses": analyses,
                   "field_rel_error_vs_fp64": field_err},
        "roofline": roofline,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    return line


def bench_n100(args, mh, W):
    """N=100 in an 80 nm lysosome, FP64 end to end, 3 periods of 2000 steps.
    One replica is a chain of 6000 dependent steps in one resident workgroup (latency:
    us per time step); 1024 replicas on their own Philox streams show the throughput of
    the same kernel."""
    a1 = W.lysosome_n100()
    ctx = mh.Context(0)
    asm = mh.Assembly(ctx, a1.pos, a1.axes, mh.params_from_material(a1.mat, mh.FP64))
    steps_per_run = a1.mat.steps_per_period * a1.mat.n_periods
    out = {}
    for R in (1, 1024):
        for _ in range(args.warmup):
            asm.run(R, seed=a1.seed)
            asm.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            asm.run(R, seed=a1.seed)
            asm.sync()
        out[R] = (time.perf_counter() - t0) / args.steps
    sar = asm.sar()
    # latency floor of a resident step: one LDS exchange and one barrier per step
    us_empty = ctx.time_empty_steps(steps_per_run)
    # the whole run is one resident launch: its duration from one event pair
    ctx.set_timing(True)
    asm.run(1024, seed=a1.seed)
    asm.sync()
    ms_k, launches = ctx.get_timing(1)
    ctx.set_timing(False)
    us_launch = ms_k * 1e3 / max(launches, 1)
    flops = FLOPS_PER_PAIR * a1.n * (a1.n - 1) * 1024 * steps_per_run   # Eq. 1 pair terms
    return {"metric": "NP·steps/s (dipolar+kMC)", "value": a1.n * 1024 * steps_per_run / out[1024],
            "unit": "NP·steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": out[1024] * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "N=100 in an 80 nm lysosome, d=12 nm, 20 mT, 100 kHz, "
                                   "3 periods x 2000 steps, FP64, 1024 replicas",
                       "us_per_time_step_one_replica": out[1] / steps_per_run * 1e6,
                       "us_per_empty_resident_step": us_empty,
                       "one_replica_step_over_empty": out[1] / steps_per_run * 1e6 / us_empty,
                       "sar_W_per_g": sar["sar"] / 1e3, "sar_se_W_per_g": sar["sar_se"] / 1e3},
            "roofline": _roof("alu", flops, us_launch, PEAK_FP64_VECTOR, "TFLOP/s",
                              "k_resident<double> (whole run; pair terms only counted)",
                              traffic=None)}


def bench_methods(args, mh, W):
    """The paper's two ways of averaging loops (Sec. III.1, Fig. 3): 5000 particles of
    20 nm on a maximally disordered cubic lattice at phi = 1 %, K = 1.3e4, Ms = 1e6,
    300 K, 40 mT, 100 kHz, 50 loops (replicas) of 2 periods (first discarded). Method 1
    changes only the axes between loops; method 2 changes the axes and the positions
    (particle i stays near lattice node i). Reports the per-particle area against the
    normalised distance from the centre after a 200-point moving average, and the rms
    scatter of the raw per-particle means about it."""
    import numpy as np
    n, loops, d, phi = 5000, 50, 20e-9, 0.01
    radius = 0.5 * d * (n / phi) ** (1.0 / 3.0)
    mat = W.Material(Ms=1e6, Keff=1.3e4, d=d, T=300.0, mu0Hmax=0.04, n_periods=2, n_discard=1)
    axes = np.concatenate([W.axes_random_3d(n, 9500 + q) for q in range(loops)])
    pos_sets = [W.place_lattice_disorder(n, radius, d, 9600 + q) for q in range(loops)]
    ctx = mh.Context(0)
    p = mh.params_from_material(mat, mh.FP32_FIELD)
    m1 = mh.Assembly(ctx, pos_sets[0], axes, p, n_axes_sets=loops)
    m2 = mh.Assembly(ctx, np.concatenate(pos_sets), axes, p, n_axes_sets=loops, n_pos_sets=loops)
    # mean positions: the lattice nodes, i.e. the mean over the position sets
    rnorm = np.linalg.norm(np.mean(pos_sets, axis=0), axis=1) / radius
    order = np.argsort(rnorm, kind="stable")
    out, walls = {}, {}
    for name, a in (("method1_axes", m1), ("method2_axes_and_positions", m2)):
        t0 = time.perf_counter()
        a.run(loops, seed=77)
        a.sync()
        walls[name] = time.perf_counter() - t0
        raw = a.sar(per_np=True)["area_per_np"][order]
        smooth = np.convolve(raw, np.ones(200) / 200, mode="valid")
        centre = raw[99:99 + smooth.shape[0]]
        x = rnorm[order][99:99 + smooth.shape[0]]
        pick = [min(int(np.searchsorted(x, v)), x.shape[0] - 1) for v in (0.2, 0.4, 0.6, 0.8, 0.9, 0.95)]
        out[name] = {"rms_scatter_about_average_Jm3": float(np.sqrt(np.mean((centre - smooth) ** 2))),
                     "mean_area_Jm3": float(raw.mean()),
                     "smoothed_area_at_r": {f"{x[i]:.2f}": float(smooth[i]) for i in pick}}
    steps = mat.steps_per_period * mat.n_periods
    line = {"metric": "NP·steps/s (dipolar+kMC)",
            "value": n * loops * steps / walls["method2_axes_and_positions"], "unit": "NP·steps/s",
            "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": walls["method2_axes_and_positions"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32 field / f64 barrier",
            "data": "synthetic",
            "config": {"workload": "averaging methods: 5000 NPs, d=20 nm, phi=1 %, 40 mT, 50 loops "
                                   "(value: method 2, one geometry per loop)",
                       "seconds": walls, **out}}
    print(json.dumps(line), flush=True)


def bench_sweep(args, mh, W):
    """Concentration sweep of large particles (Sec. III.2-3, the d -> infinity case): 3000
    particles on a maximally disordered cubic lattice, random 3-D axes (8 axis sets as
    replicas), Ms = 1e6 A/m, K = 1.3e4 J/m^3, T = 0, 40 mT, 100 kHz, 2 periods of 2000
    steps (first discarded), volume fractions 0.01-30 %, all assemblies in one batch.
    Reports the dimensionless area A/K against the dimensionless concentration
    mu0 Ms^2 phi / K."""
    import numpy as np
    n, sets, d = 3000, 8, 20e-9
    phis = [1e-4, 1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.3]
    Ms, K = 1e6, 1.3e4
    ctx = mh.Context(0)
    asms = []
    for q, phi in enumerate(phis):
        radius = 0.5 * d * (n / phi) ** (1.0 / 3.0)
        pos = W.place_lattice_disorder(n, radius, d, 8000 + q)
        axes = np.concatenate([W.axes_random_3d(n, 8100 + 10 * q + s_) for s_ in range(sets)])
        mat = W.Material(Ms=Ms, Keff=K, d=d, T=0.0, mu0Hmax=0.04, n_periods=2, n_discard=1)
        asms.append(mh.Assembly(ctx, pos, axes, mh.params_from_material(mat, mh.FP32_FIELD),
                                n_axes_sets=sets))
    steps_per_run = 2 * 2000

    def one_run():
        mh.run_batch(asms, [sets] * len(asms), [9000 + q for q in range(len(asms))])
        for a in asms:
            a.sync()
        return [a.sar() for a in asms]

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_run()
    t1 = time.perf_counter()
    wall = t1 - t0
    mu0 = 4e-7 * np.pi
    curve = [{"phi": phi, "mu0_Ms2_phi_over_K": mu0 * Ms ** 2 * phi / K,
              "A_over_K": r["area"] / K, "se": r["area_se"] / K} for phi, r in zip(phis, res)]
    line = {"metric": "NP·steps/s (dipolar+kMC)",
            "value": n * sets * len(phis) * steps_per_run * args.steps / wall, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 field / f64 barrier", "data": "synthetic",
            "config": {"workload": "concentration sweep: 3000 NPs, lattice + maximal disorder, "
                                   "T=0, Ms=1e6, K=1.3e4, 40 mT, 8 axis sets, phi 0.01-30 %",
                       "A_over_K_vs_dimensionless_concentration": curve}}
    print(json.dumps(line), flush=True)


def bench_figs(args, mh, W):
    """Parameter sweeps of Sec. III.2-4 as one batch of assemblies, giving the curves of
    Fig. 4(a) (area against phi for d -> infinity at T = 0, d = 20 nm, d = 9 nm and
    K = T = 0), Fig. 6(a) (d = 20 nm at 40 mT, 1 T and 7 mT), Fig. 7 (A/K against
    mu0 Ms^2 phi / K for an anisotropy and a magnetisation series at T = 0, with
    mu0 Hmax / K fixed in the anisotropy series) and Fig. 10 (9 nm particles, lysosomes
    of 10 to 3000). Defaults are the paper's (Ms = 1e6 A/m, K = 13000 J/m^3, T = 300 K,
    40 mT, 100 kHz, nu0 = 1e10 Hz); 3000 particles on a maximally disordered cubic
    lattice, 8 random 3-D axis sets per point as replicas (the paper's averaging over
    axis orientations), 2 periods of 2000 steps with the first discarded. The phi
    points are those of Fig. 5 (0.01-30 %); points that the lattice cannot place (10
    and 100 particles at 30 %) are skipped. The dilute end of each finite-size series
    is set against the deterministic loop of the same particles without interactions
    (mean-magnetisation kernel, same axis sets and amplitudes), and the T = 0 series
    against the Stoner-Wohlfarth value 1.977 (at mu0 Ms^2 phi / K <= 0.02 interactions
    are negligible)."""
    import numpy as np
    mu0 = 4e-7 * np.pi
    phis = [1e-4, 5e-4, 1e-3, 3e-3, 6e-3, 1e-2, 2e-2, 3e-2, 0.1, 0.3]
    sets = 8
    base = dict(Ms=1e6, Keff=1.3e4, T=300.0, f=1e5, mu0Hmax=0.04, n_periods=2, n_discard=1)
    # (name, figures, particles, d, overrides, per-replica amplitudes or None)
    series = [("d_inf_T0", "4a,7", 3000, 20e-9, dict(T=0.0), None),
              ("d20nm", "4a,6a", 3000, 20e-9, {}, (0.04, 1.0, 0.007)),
              ("d9nm", "4a,10", 3000, 9e-9, {}, None),
              ("K0_T0", "4a", 3000, 20e-9, dict(Keff=0.0, T=0.0), None)]
    for K in (6e3, 1e5, 1e6):
        series.append((f"T0_K{K:g}", "7", 3000, 20e-9,
                       dict(T=0.0, Keff=K, mu0Hmax=0.04 * K / 1.3e4), None))
    for Ms in (7e5, 1.7e6):
        series.append((f"T0_Ms{Ms:g}", "7", 3000, 20e-9, dict(T=0.0, Ms=Ms), None))
    for N in (10, 100, 1000):
        series.append((f"d9nm_N{N}", "10", N, 9e-9, {}, None))
    ctx = mh.Context(0)
    asms, meta, Rs, skipped = [], [], [], []
    q = 0
    for si, (name, figs, n, d, over, amps) in enumerate(series):
        kw = dict(base, d=d, **over)
        for phi in phis:
            q += 1
            radius = 0.5 * d * (n / phi) ** (1.0 / 3.0)
            try:
                pos = W.place_lattice_disorder(n, radius, d, 9000 + q)
            except RuntimeError:
                skipped.append({"series": name, "phi": phi})
                continue
            axes = np.concatenate([W.axes_random_3d(n, 9500 + 10 * si + k) for k in range(sets)])
            a = mh.Assembly(ctx, pos, axes, mh.Params.make(mh.FP32_FIELD, **kw), n_axes_sets=sets)
            R = sets
            if amps:
                a.set_replica_fields(list(amps))
                R = sets * len(amps)
            asms.append(a)
            Rs.append(R)
            meta.append((si, phi, n, kw))
    steps_per_run = 2 * 2000
    seeds = [12000 + i for i in range(len(asms))]

    def one_run():
        mh.run_batch(asms, Rs, seeds)
        for a in asms:
            a.sync()

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_run()
    wall = time.perf_counter() - t0
    npsteps = sum(m[2] * R for m, R in zip(meta, Rs)) * steps_per_run * args.steps
    # curves
    out = {}
    for (si, phi, n, kw), a, R in zip(meta, asms, Rs):
        name, figs, _, d, over, amps = series[si]
        ra = a.replica_areas()
        groups = [(f"{h * 1e3:g} mT", ra[k::len(amps)]) for k, h in enumerate(amps)] if amps \
            else [("", ra)]
        for label, vals in groups:
            key = name + (f"_{label.replace(' ', '')}" if label else "")
            A = float(vals.mean())
            se = float(vals.std(ddof=1) / np.sqrt(len(vals)))
            pt = {"phi": phi, "area_Jm3": A, "se": se, "sar_W_per_g": A * kw["f"] / 5200.0 / 1e3}
            if kw["Keff"] > 0:
                pt["mu0_Ms2_phi_over_K"] = mu0 * kw["Ms"] ** 2 * phi / kw["Keff"]
                pt["A_over_K"] = A / kw["Keff"]
            out.setdefault(key, {"figures": figs, "n": n, "d_nm": d * 1e9, "points": []})
            out[key]["points"].append(pt)
    # dilute-limit checks
    checks = {}
    for si, (name, figs, n, d, over, amps) in enumerate(series):
        kw = dict(base, d=d, **over)
        first = next(((m, a) for m, a in zip(meta, asms) if m[0] == si), None)
        if first is None:
            continue
        (_, phi0, _, _), a0 = first
        if kw["T"] > 0 and kw["Keff"] > 0:
            pos = W.place_lattice_disorder(n, 0.5 * d * (n / phi0) ** (1 / 3), d, 1)
            axes = np.concatenate([W.axes_random_3d(n, 9500 + 10 * si + k) for k in range(sets)])
            b = mh.Assembly(ctx, pos, axes, mh.Params.make(mh.FP64, **dict(kw, interactions=0)),
                            n_axes_sets=sets)
            R = sets
            if amps:
                b.set_replica_fields(list(amps))
                R = sets * len(amps)
            b.run_mean_loop(R)
            b.sync()
            det = b.replica_areas()
            b.close()
            ra = a0.replica_areas()
            for k, h in enumerate(amps or (kw["mu0Hmax"],)):
                sl = slice(k, None, len(amps)) if amps else slice(None)
                kmc_v, det_v = ra[sl], det[sl]
                se = float(kmc_v.std(ddof=1) / np.sqrt(len(kmc_v)))
                checks[f"{name}_{h * 1e3:g}mT"] = {
                    "phi": phi0, "kmc_area": float(kmc_v.mean()), "se": se,
                    "no_interaction_area": float(det_v.mean()),
                    "z": float((kmc_v.mean() - det_v.mean()) / max(se, 1e-12))}
        elif kw["T"] == 0 and kw["Keff"] > 0:
            ra = a0.replica_areas()
            checks[name] = {"phi": phi0, "A_over_K": float(ra.mean() / kw["Keff"]),
                            "stoner_wohlfarth": 1.977,
                            "mu0_Ms2_phi_over_K": mu0 * kw["Ms"] ** 2 * phi0 / kw["Keff"]}
    line = {"metric": "NP·steps/s (dipolar+kMC)", "value": npsteps / wall, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 field / f64 barrier", "data": "synthetic",
            "config": {"workload": f"parameter sweeps of Figs. 4a/6a/7/10: {len(asms)} assemblies "
                                   f"in one batch, {sum(Rs)} replicas, 2 periods x 2000 steps",
                       "curves": out, "dilute_limit_checks": checks, "skipped": skipped}}
    print(json.dumps(line), flush=True)


def bench_master(args, mh, W):
    """Deterministic mean-magnetisation loops (non-interacting particles, the paper's
    validation method): 10 000 particles with random 3-D axes, 8 axis sets run together,
    material of the N = 5000 lysosome at 20 mT, 100 kHz, --periods periods of 2000 steps. One launch per
    run; value counts particle-steps of the weighted two-well state."""
    import numpy as np
    n, sets = 10000, 8
    axes = np.concatenate([W.axes_random_3d(n, 7000 + q) for q in range(sets)])
    pos = W.place_lattice_disorder(n, 400e-9, 12e-9, 7100)   # unused without interactions
    mat = W.Material(mu0Hmax=0.02, n_periods=args.periods, n_discard=min(1, args.periods - 1),
                     interactions=0)
    ctx = mh.Context(0)
    asm = mh.Assembly(ctx, pos, axes, mh.params_from_material(mat, mh.FP64), n_axes_sets=sets)
    steps_per_run = mat.steps_per_period * mat.n_periods

    def one_run():
        asm.run_mean_loop(sets)
        asm.sync()
        return asm.sar()

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_run()
    t1 = time.perf_counter()
    ctx.set_timing(True)
    one_run()
    ms_k, launches = ctx.get_timing(5)
    ctx.set_timing(False)
    wall = t1 - t0
    line = {"metric": "NP·steps/s (mean-magnetisation loop, no interactions)",
            "value": n * sets * steps_per_run * args.steps / wall, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"mean loop: N={n}, {sets} axis sets, 20 mT, 100 kHz, "
                                   f"{args.periods} periods x 2000 steps",
                       "sar_W_per_g": res["sar"] / 1e3, "sar_spread_W_per_g": res["sar_se"] / 1e3},
            "kernel": {"name": "k_master", "ms_per_launch": ms_k / max(launches, 1),
                       "launches": launches}}
    print(json.dumps(line), flush=True)


def bench_served(args, mh, W):
    """Serving (continuous batching): loop-simulation requests with N log-uniform in
    [100, 8000], radius U(80,300) nm, phi U(1,20) %, f log-uniform in [1e5, 1e6] Hz,
    Hmax U(5,50) mT, 3-10 periods (one discarded), each run in rounds of replicas until
    2 SE <= 1 % of its area (no absolute floor) or --max-replicas. Both engines serve the
    same request stream: the plain FP32 N-body kernels and the interaction-matrix form on
    MFMA. For each engine, the first --sat-requests requests are submitted at once to
    measure its saturated request rate (they also warm it up); then, for each factor of
    --rates, --requests further requests arrive as a Poisson stream at that factor of the
    plain engine's saturated rate, on a fresh server. Reported per engine and rate:
    kept loops/s, p50/p99 request latency, and the achieved 2 SE / area."""
    import numpy as np
    rates = [float(x) for x in args.rates.split(",") if x.strip()]  # "": saturation only
    n_sat, n_rate = args.sat_requests, args.requests
    reqs = W.request_stream(count=n_sat + n_rate * len(rates), seed=1005, rate_hz=1.0)
    geo = []
    for q in reqs:
        pos = W.place_random(q["n"], q["R"], q["d"], q["seed"])
        axes = W.axes_random_3d(q["n"], q["seed"] + 1)
        geo.append((pos, axes, q))

    def params(prec, q):
        return mh.Params.make(prec, Ms=4e5, Keff=1.3e4, d=q["d"], T=300.0, tau0=1e-10,
                              rho=5200.0, f=q["f"], mu0Hmax=q["H"], steps_per_period=2000,
                              n_periods=q["P"], n_discard=1)

    ctx = mh.Context(0)

    def serve(prec, items, gaps, label):
        srv = mh.Server(ctx, 200 << 30)
        ids, t0 = [], time.perf_counter()
        for (pos, axes, q), ta in zip(items, gaps):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.0005)
            ids.append(srv.submit(pos, axes, params(prec, q), seed=q["seed"], target_rel_err=0.01,
                                  abs_err_floor=0.0, min_replicas=64,
                                  max_replicas=args.max_replicas))
            print(f"served {label}: request {len(ids) - 1} submitted (N={q['n']}, "
                  f"{q['P']} periods)", file=sys.stderr, flush=True)
        out, seen = {}, {}
        while len(out) < len(ids):
            for k, i in enumerate(ids):
                if i not in out:
                    r = srv.poll(i)
                    if r is not None:
                        out[i] = r
                        print(f"served {label}: {len(out)}/{len(ids)} done, {r['replicas']} "
                              f"replicas, {(r['done_ns'] - r['submit_ns']) / 1e9:.2f} s",
                              file=sys.stderr, flush=True)
                    else:
                        done_r = srv.progress(i)
                        if done_r != seen.get(i, 0):   # a round of this request finished
                            seen[i] = done_r
                            print(f"served {label}: request {k} at {done_r} replicas",
                                  file=sys.stderr, flush=True)
            time.sleep(0.002)
        srv.close()
        res = [out[i] for i in ids]
        first = min(r["submit_ns"] for r in res)
        last = max(r["done_ns"] for r in res)
        lat = np.array([(r["done_ns"] - r["submit_ns"]) / 1e9 for r in res])
        rel = np.array([2 * r["area_se"] / max(abs(r["area_Jm3"]), 1e-300) for r in res])
        loops = sum(r["loops"] for r in res)
        npsteps = sum(q["n"] * 2000 * q["P"] * r["replicas"] for (_, _, q), r in zip(items, res))
        span = (last - first) / 1e9
        return {"requests": len(res), "seconds": span, "loops_per_s": loops / span,
                "np_steps_per_s": npsteps / span,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "two_se_over_area_median": float(np.median(rel)),
                "two_se_over_area_max": float(rel.max()),
                "fraction_within_1pct": float(np.mean(rel <= 0.01 + 1e-12)),
                "replicas_median": float(np.median([r["replicas"] for r in res])),
                "replicas_max": int(max(r["replicas"] for r in res)),
                "status_ok": all(r["status"] == 0 for r in res)}

    all_engines = {"plain_fp32": mh.FP32_FIELD, "matrix_bf16x3": mh.BF16X3_WM}
    engines = {k: v for k, v in all_engines.items() if k.split("_")[0] in args.engines.split(",")}
    out = {name: {} for name in engines}
    for name, prec in engines.items():
        if n_sat > 0:  # --sat-requests 0: rate phases only, at the given --lambda0
            sat = serve(prec, geo[:n_sat], [0.0] * n_sat, f"{name} saturation")
            out[name]["saturated"] = dict(sat, req_per_s=n_sat / sat["seconds"])
    # arrival rates are factors of the plain engine's saturated rate (measured here, or
    # given when the engines run in separate processes)
    if not args.lambda0 and "saturated" not in out.get("plain_fp32", {}):
        raise SystemExit("served: give --lambda0 when the plain engine's saturation is not run")
    lam0 = args.lambda0 or out["plain_fp32"]["saturated"]["req_per_s"]
    rng = np.random.default_rng(77)
    for k, fct in enumerate(rates):
        items = geo[n_sat + k * n_rate:n_sat + (k + 1) * n_rate]
        gaps = np.cumsum(rng.exponential(1.0 / (fct * lam0), size=len(items)))
        gaps -= gaps[0]
        for name, prec in engines.items():
            out[name][f"rate_{fct:g}x"] = dict(serve(prec, items, gaps, f"{name} {fct:g}x"),
                                               arrival_req_per_s=fct * lam0)
    eng = out.get("matrix_bf16x3") or out["plain_fp32"]
    main = eng.get("rate_0.7x") or eng.get("saturated") or next(iter(eng.values()))
    return {"metric": "served loops/s; p50/p99 request latency at SAR err<=1%",
            "value": main["loops_per_s"], "unit": "loops/s", "n_gpus": 1,
            "steps": n_rate * len(rates), "warmup": n_sat,
            "ms_per_step": main["seconds"] / max(main["requests"], 1) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16x3 mfma / f64 barrier (value); f32 field / f64 barrier (plain)",
            "data": "synthetic",
            "config": {"workload": f"served request stream: {n_sat} saturation requests per engine, "
                                   f"then {n_rate} Poisson arrivals at each of {rates} x the plain "
                                   f"engine's saturated rate ({lam0:.4g} req/s); value: "
                                   f"{'matrix' if 'matrix_bf16x3' in out else 'plain'} engine "
                                   f"at 0.7x",
                       "max_replicas": args.max_replicas, "target_two_se_over_area": 0.01,
                       "engines": out}}


def bench_uneven256(args, mh, W):
    """Batched uneven assemblies: 256 lysosomes with R ~ U(100,250) nm, phi ~ U(1,20) %,
    d ~ U(10,16) nm, K ~ U(0.8,2)e4, Hmax ~ U(5,40) mT, N in [200, 8000], one replica
    each, FP32 field, run together."""
    import numpy as np
    work = W.uneven_batch(count=args.assemblies, n_periods=args.periods)
    ctx = mh.Context(0)
    tune = None
    if not args.no_tune:
        # launch shapes from the autotuner: one representative N (the median) per
        # particle-count bucket present in the batch, one replica each
        ns = np.array(sorted(w.n for w in work if w.n > 256))
        buckets = 2 ** np.ceil(np.log2(np.maximum(ns, 256)))
        sizes = [int(np.median(ns[buckets == b])) for b in np.unique(buckets)]
        t0 = time.perf_counter()
        ctx.autotune(mh.FP32_FIELD, sizes, [1])
        tune = {"sizes": sizes, "seconds": time.perf_counter() - t0}
    asms = [mh.Assembly(ctx, w.pos, w.axes, mh.params_from_material(w.mat, mh.FP32_FIELD))
            for w in work]
    seeds = [w.seed for w in work]
    npsteps = sum(w.n * w.mat.steps_per_period * w.mat.n_periods for w in work)
    steps_per_run = max(w.mat.steps_per_period * w.mat.n_periods for w in work)

    def one_run():
        mh.run_batch(asms, [1] * len(asms), seeds)
        for a in asms:
            a.sync()
        return [a.sar()["sar"] for a in asms]

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sars = one_run()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = npsteps * args.steps / wall
    us_step = wall / (args.steps * steps_per_run) * 1e6
    tiled = [a for a, w in zip(asms, work) if w.n > 256]
    us_field = mh.time_kernels(tiled, 0, 50, 10)
    us_update = mh.time_kernels(tiled, 3, 50, 10)
    pairs = sum(w.n * (w.n - 1) for w in work if w.n > 256)
    return {"metric": "NP·steps/s (dipolar+kMC)", "value": value, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 field / f64 barrier", "data": "synthetic",
            "config": {"workload": f"{len(work)} uneven assemblies, N {min(w.n for w in work)}"
                                   f"-{max(w.n for w in work)}, {args.periods} periods x 2000 steps",
                       "n_particles_total": sum(w.n for w in work),
                       "us_per_time_step": us_step,
                       "sar_W_per_g_median": float(sorted(sars)[len(sars) // 2]) / 1e3,
                       "autotuned_shapes": tune},
            "roofline": _roof("alu", FLOPS_PER_PAIR * pairs, us_field, PEAK_FP32_VECTOR,
                              "TFLOP/s", "k_field<float> (all field launches of one step)",
                              traffic=None, update_us_per_step=us_update,
                              kernels_over_step=(us_field + us_update) / us_step,
                              timing="graph replay of 50 steps x 10 on the timed run's plan "
                                     "(tiled members; the resident members run in one "
                                     "launch beside them)")}


def bench_replicas512(args, mh, W):
    """Replica-batched form: N=4096 in a 200 nm lysosome at phi=10 %, one axis set per
    replica, R replicas on independent Philox streams; W.M on MFMA (replicas512) or the plain
    FP32 N-body kernels on the same replicas (replicas512plain)."""
    R = args.replicas
    a4 = W.replica_batch_n4096(n_axes_sets=R)
    a4.mat.n_periods = args.periods
    a4.mat.n_discard = min(a4.mat.n_discard, args.periods - 1)
    wm = args.workload == "replicas512"
    prec = mh.BF16X3_WM if wm else mh.FP32_FIELD
    ctx = mh.Context(0)
    asm = mh.Assembly(ctx, a4.pos, a4.axes, mh.params_from_material(a4.mat, prec), n_axes_sets=R)
    steps_per_run = a4.mat.steps_per_period * a4.mat.n_periods

    def one_run():
        asm.run(R, seed=a4.seed)
        asm.sync()
        return asm.sar()

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_run()
    t1 = time.perf_counter()
    wall = t1 - t0
    n = a4.n
    value = n * R * steps_per_run * args.steps / wall
    us_step = wall / (args.steps * steps_per_run) * 1e6
    # field error of this form on replica 0's final moments, against the FP64 field
    # kernel (which the parity tests hold within 1e-13 of the FP64 oracle): relative
    # Frobenius norm and the largest per-particle error over the rms field
    rel, mx = asm.field_error(0)
    field_err = {"rel_frobenius": rel, "max_over_rms": mx}
    us_k = mh.time_kernels([asm], 2 if wm else 0, 20, 10)
    us_u = mh.time_kernels([asm], 4 if wm else 3, 20, 10)
    if wm:
        alg = 2.0 * (3 * n) ** 2 * R          # one W.M product per step
        roof = _roof("mfma", alg, us_k, PEAK_BF16_MFMA, "TFLOP/s", "k_wm_gemm", traffic=None,
                     mfma_utilisation_executed=3 * alg / (us_k * 1e-6) / PEAK_BF16_MFMA,
                     update_us_per_step=us_u, kernels_over_step=(us_k + us_u) / us_step)
    else:
        alg = FLOPS_PER_PAIR * n * (n - 1) * R
        roof = _roof("alu", alg, us_k, PEAK_FP32_VECTOR, "TFLOP/s", "k_field<float>",
                     traffic=None, update_us_per_step=us_u,
                     kernels_over_step=(us_k + us_u) / us_step)
    return {"metric": "NP·steps/s (dipolar+kMC)", "value": value, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "bf16x3 mfma / f64 barrier" if wm else "f32 field / f64 barrier",
            "data": "synthetic",
            "config": {"workload": f"replica batch ({args.workload}): N={n}, R={R} replicas, 200 nm, "
                                   f"phi=10%, d={a4.mat.d * 1e9:.2f} nm, 20 mT, {args.periods} periods",
                       "us_per_time_step": us_step,
                       "sar_W_per_g": res["sar"] / 1e3, "sar_se_W_per_g": res["sar_se"] / 1e3,
                       "field_error_vs_fp64": field_err},
            "roofline": roof}


if __name__ == "__main__":
    main()
