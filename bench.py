"""Throughput of the kMC hysteresis hot path on one MI355X, in NP.steps/s.

Workload (default, the paper-scale plain form): one lysosome of radius 250 nm holding
5000 hard spheres of 12 nm (phi = 6.9 %), random 3-D easy axes, Ms = 4e5 A/m,
K = 1.3e4 J/m^3, T = 300 K, tau0 = 1e-10 s, 100 kHz, at three field amplitudes
(10, 20, 40 mT) run together as one batch of three assemblies, 5 periods of 2000 steps
(first discarded). Dipolar sum in FP32, per-particle barrier step and area in FP64.

One bench step = one complete run of the batch (all 3 x 5 x 2000 time steps, each with
every part of the path: dipolar field, Stoner-Wohlfarth extrema, switching draw, area
accumulation, then the SAR reduction). value = NP.steps executed / wall time, with the
inputs already resident in device memory.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak, FLOP/s
FLOPS_PER_PAIR = 30             # Eq. 1 pair term as evaluated


def cpu_baseline(assemblies, budget_s=15.0):
    """The FP64 oracle on the host: a bounded number of steps of the same workload."""
    import numpy as np
    from oracle import kmc
    a = assemblies[1]
    p = kmc.Params.from_dict(a.mat.as_dict())
    m = kmc.initial_moments(a.axes)
    t0 = time.perf_counter()
    k = 0
    while True:
        m, _ = kmc.step(a.pos, a.axes, m, k, p, a.seed, 0)
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 200:
            break
    dt = time.perf_counter() - t0
    return {"value": a.n * k / dt, "unit": "NP·steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} steps of the 20 mT assembly (N={a.n}), single-threaded numpy FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--periods", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c4plain"])
    ap.add_argument("--assemblies", type=int, default=256)
    ap.add_argument("--replicas", type=int, default=512)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path is a single-device build; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import paper_1407_2737_amd as mh
    from paper_1407_2737_amd import workloads as W

    if args.workload == "c3":
        return bench_c3(args, mh, W)
    if args.workload != "c2":
        return bench_c4(args, mh, W)

    amps = (0.010, 0.020, 0.040)
    work = [W.config2(mu0Hmax=h, n_periods=args.periods) for h in amps]
    ctx = mh.Context(0)
    asms = [mh.Assembly(ctx, w.pos, w.axes, mh.params_from_material(w.mat, mh.FP32_FIELD))
            for w in work]
    seeds = [w.seed + q for q, w in enumerate(work)]
    n_total = sum(w.n for w in work)
    steps_per_run = work[0].mat.steps_per_period * work[0].mat.n_periods

    def one_run():
        mh.run_batch(asms, [1] * len(asms), seeds)
        out = []
        for a in asms:
            a.sync()
            out.append(a.sar())
        return out

    for _ in range(args.warmup):
        one_run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_run()
    t1 = time.perf_counter()
    # kernel durations: the timed runs replay captured graphs, which cannot carry
    # per-launch events; one more run of the same plan launches the same kernels one by
    # one, each bracketed by HIP events on the library's stream
    ctx.set_timing(True)
    one_run()
    ms_kernel, launches = ctx.get_timing(0)
    ms_update, launches_u = ctx.get_timing(3)
    ctx.set_timing(False)
    wall = t1 - t0
    np_steps = n_total * steps_per_run * args.steps
    value = np_steps / wall
    avg_launch_s = ms_kernel / 1e3 / max(launches, 1)
    pairs_per_launch = sum(w.n * (w.n - 1) for w in work)
    achieved = FLOPS_PER_PAIR * pairs_per_launch / avg_launch_s
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                "kernel": "k_field<float>", "avg_launch_us": avg_launch_s * 1e6,
                "launches": launches,
                "update_kernel_avg_us": ms_update * 1e3 / max(launches_u, 1)}
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
        "config": {"workload": "config2: N=5000 in a 250 nm lysosome, d=12 nm (phi=6.9%), "
                               "random 3-D axes, 10/20/40 mT batched, 100 kHz, "
                               f"{args.periods} periods x 2000 steps",
                   "n_particles_total": n_total, "steps_per_run": steps_per_run,
                   "sar_W_per_g": [r[0]["sar"] / 1e3 for r in [[x] for x in res]]},
        "roofline": roofline,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(work)
    print(json.dumps(line), flush=True)


def bench_c3(args, mh, W):
    """Batched uneven assemblies: 256 lysosomes with R ~ U(100,250) nm, phi ~ U(1,20) %,
    d ~ U(10,16) nm, K ~ U(0.8,2)e4, Hmax ~ U(5,40) mT, N in [200, 8000], one replica
    each, FP32 field, run together."""
    work = W.config3(count=args.assemblies, n_periods=args.periods)
    ctx = mh.Context(0)
    asms = [mh.Assembly(ctx, w.pos, w.axes, mh.params_from_material(w.mat, mh.FP32_FIELD))
            for w in work]
    seeds = [w.seed for w in work]
    npsteps = sum(w.n * w.mat.steps_per_period * w.mat.n_periods for w in work)

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
    ctx.set_timing(True)
    one_run()
    ms_k, launches = ctx.get_timing(0)
    ms_u, lu = ctx.get_timing(3)
    ms_r, lr = ctx.get_timing(1)
    ctx.set_timing(False)
    wall = t1 - t0
    value = npsteps * args.steps / wall
    pairs = sum(w.n * (w.n - 1) for w in work if w.n > 256)
    avg = ms_k / 1e3 / max(launches, 1)
    roof = {"bound": "alu", "achieved": FLOPS_PER_PAIR * pairs / avg / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": FLOPS_PER_PAIR * pairs / avg / PEAK_FP32_VECTOR, "traffic": None,
            "kernel": "k_field<float>", "avg_launch_us": avg * 1e6, "launches": launches,
            "update_kernel_avg_us": ms_u * 1e3 / max(lu, 1), "resident_ms": ms_r}
    line = {"metric": "NP·steps/s (dipolar+kMC)", "value": value, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 field / f64 barrier", "data": "synthetic",
            "config": {"workload": f"config3: {len(work)} uneven assemblies, N {min(w.n for w in work)}"
                                   f"-{max(w.n for w in work)}, {args.periods} periods x 2000 steps",
                       "n_particles_total": sum(w.n for w in work),
                       "sar_W_per_g_median": float(sorted(sars)[len(sars) // 2]) / 1e3},
            "roofline": roof}
    print(json.dumps(line), flush=True)


def bench_c4(args, mh, W):
    """Replica-batched form: N=4096 in a 200 nm lysosome at phi=10 %, one axis set per
    replica, R replicas on independent Philox streams; W.M on MFMA (c4) or the plain
    FP32 N-body kernels on the same replicas (c4plain)."""
    R = args.replicas
    a4 = W.config4(n_axes_sets=R)
    a4.mat.n_periods = args.periods
    a4.mat.n_discard = min(a4.mat.n_discard, args.periods - 1)
    prec = mh.BF16X3_WM if args.workload == "c4" else mh.FP32_FIELD
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
    ctx.set_timing(True)
    one_run()
    kind = 2 if args.workload == "c4" else 0
    ms_k, launches = ctx.get_timing(kind)
    ms_u, lu = ctx.get_timing(4 if args.workload == "c4" else 3)
    ctx.set_timing(False)
    wall = t1 - t0
    n = a4.n
    value = n * R * steps_per_run * args.steps / wall
    avg = ms_k / 1e3 / max(launches, 1)
    if args.workload == "c4":
        alg = 2.0 * (3 * n) ** 2 * R          # one W.M product per step
        roof = {"bound": "mfma", "achieved": alg / avg / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                "frac": alg / avg / 2.5e15, "traffic": None, "kernel": "k_wm_gemm",
                "avg_launch_us": avg * 1e6, "launches": launches,
                "mfma_utilisation_executed": 3 * alg / avg / 2.5e15,
                "update_kernel_avg_us": ms_u * 1e3 / max(lu, 1)}
    else:
        alg = FLOPS_PER_PAIR * n * (n - 1) * R
        roof = {"bound": "alu", "achieved": alg / avg / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": alg / avg / PEAK_FP32_VECTOR, "traffic": None,
                "kernel": "k_field<float>", "avg_launch_us": avg * 1e6, "launches": launches,
                "update_kernel_avg_us": ms_u * 1e3 / max(lu, 1)}
    line = {"metric": "NP·steps/s (dipolar+kMC)", "value": value, "unit": "NP·steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "bf16x3 mfma / f64 barrier" if args.workload == "c4" else "f32 field / f64 barrier",
            "data": "synthetic",
            "config": {"workload": f"config4 ({args.workload}): N={n}, R={R} replicas, 200 nm, "
                                   f"phi=10%, d={a4.mat.d * 1e9:.2f} nm, 20 mT, {args.periods} periods",
                       "sar_W_per_g": res["sar"] / 1e3, "sar_se_W_per_g": res["sar_se"] / 1e3},
            "roofline": roof}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
