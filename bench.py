"""Benchmark: Q(f,f) evaluations per second for the 3D N=32^3 workload on one MI355X.

Workload (the paper's 3D BKW test, Sec. 5.2, at the size of the headline metric):
3D, N = 32 modes per dimension (32768 coefficients), logarithmic map with
S = 5, Maxwell molecules B = 1/(4 pi), 64 sphere directions (8 Gauss-Legendre
polar x 8 uniform azimuthal nodes), initial data the closed-form 3D BKW
solution at t0 = 6.5, classical RK4 with dt = 0.1.

One step = one RK4 step (four evaluations of Q through the whole hot path:
synthesis, loss, pair-orbit sums, spreading, cosine transform, combination)
followed by the FP64 moment projection of the new state.  `value` is
evaluations per second of the FP64 path (4 per step); the FP32 variant is
timed the same way and reported with its rel-L2 against the FP64 path.

Prints one JSON line.  `--gpus N` with N > 1 exits: this benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q(f,f) evals/s, 3D N=32^3: FP64 plain vs FP32/batched/surrogate at stated rel-L2"
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}  # MI355X vector peaks, FLOP/s
N, S, T0, DT = 32, 5.0, 6.5, 0.1
N_THETA, N_PHI = 8, 8
KERNEL_SOURCE = os.path.join(ROOT, "paper_2105_08806_amd", "csrc", "pgc_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_plan(pgc, precision):
    return pgc.Plan(dim=3, n_modes=N, scale=S, map=pgc.MAP_LOG, kernel=pgc.KERNEL_MAXWELL,
                    sphere=pgc.SPHERE_PRODUCT_3D, n_theta=N_THETA, n_phi=N_PHI,
                    precision=precision)


def time_variant(torch, pgc, inputs, precision, steps, warmup):
    t0 = time.time()
    plan = make_plan(pgc, precision)
    f_nodes = inputs.bkw_f(T0, plan.interior_velocities())
    c = plan.project(f_nodes)
    torch.cuda.synchronize()
    log("plan %s ready in %.1f s: W=%d, %d points, %d bin items, %.1f GB" % (
        "fp64" if precision == pgc.FP64 else "fp32", time.time() - t0, plan.info.kernel_width,
        plan.info.n_points, plan.info.n_bin_items, plan.info.workspace_bytes / 1e9))
    state = c.double().contiguous()
    q0 = plan.coeffs_to_q(c)  # Q at t0 for the accuracy comparison
    for _ in range(warmup):
        plan.rk4(state, DT, 1)
        plan.moments(state.to(plan.dtype))
    torch.cuda.synchronize()
    plan.set_profiling(True)
    plan.stage_times()  # reset
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    moms = None
    for k in range(steps):
        plan.rk4(state, DT, 1)
        moms = plan.moments(state.to(plan.dtype))
        log("  step %d/%d done" % (k + 1, steps))
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    stages, calls = plan.stage_times()
    plan.set_profiling(False)
    out = dict(ms=ms, stages=stages, calls=calls, q0=q0.double().cpu().numpy(),
               moments=moms.cpu().numpy().tolist(), info=plan.info)
    plan.close()
    return out


def traffic_for(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken from the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    entry = rec.get(kernel_tag)
    if not entry or entry.get("kernel_source_sha256") != sha:
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(inputs, budget_s=15.0):
    """The CPU oracle (FP64, all host cores) on a bounded sample of the same
    workload: the gain of the first k collision units (s, i), scaled to
    evaluations per second of the full operator."""
    import numpy as np
    import oracle as O
    sg, sw = O.sphere_product_rule(N_THETA, N_PHI)
    p = O.Problem(3, N, S, 0, sphere=sg, sphere_w=sw)
    c = p.project(inputs.bkw_f(T0, p.interior_velocities()))
    n_units = len(sw) * (N - 1) ** 3
    k = 16
    t = time.time()
    p.gain_units(c, 0, k)
    dt = time.time() - t
    if dt < budget_s / 4:
        k = int(min(n_units, max(k, k * budget_s / max(dt, 1e-3) * 0.8)))
        t = time.time()
        p.gain_units(c, 0, k)
        dt = time.time() - t
    per_eval = dt * n_units / k
    return {"value": 1.0 / per_eval, "unit": "evals/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": "gain of %d of %d collision units (s, i) of the same 3D N=32 workload, "
                      "%.1f s, scaled to one full evaluation (%.0f s)" % (k, n_units, dt, per_eval)}


def bkw_curve(torch, pgc, inputs, np, steps=20):
    """3D BKW: RK4 from t = 6.5 with dt = 0.1 for `steps` steps in FP64 and FP32.
    Prints, per step, the rel-L2 distance of each state from the projection of
    the exact BKW solution at that time, and of the FP32 state from the FP64
    one (one JSON object per step)."""
    plans, states = {}, {}
    for prec in (pgc.FP64, pgc.FP32):
        plans[prec] = make_plan(pgc, prec)
        states[prec] = plans[prec].project(inputs.bkw_f(T0, plans[prec].interior_velocities())).double()
    V = plans[pgc.FP64].interior_velocities()
    for k in range(1, steps + 1):
        for prec in (pgc.FP64, pgc.FP32):
            plans[prec].rk4(states[prec], DT, 1)
        t = T0 + k * DT
        exact = plans[pgc.FP64].project(inputs.bkw_f(t, V)).cpu().numpy()
        s64 = states[pgc.FP64].cpu().numpy()
        s32 = states[pgc.FP32].cpu().numpy()
        nx = np.linalg.norm(exact)
        print(json.dumps({"step": k, "t": round(t, 6),
                          "fp64_vs_exact": float(np.linalg.norm(s64 - exact) / nx),
                          "fp32_vs_exact": float(np.linalg.norm(s32 - exact) / nx),
                          "fp32_vs_fp64": float(np.linalg.norm(s32 - s64) / np.linalg.norm(s64))}),
              flush=True)
    for p in plans.values():
        p.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp32-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["bench", "profile", "copy", "bkw"], default="bench",
                    help="profile: two evaluations per precision (for rocprofv3); "
                         "copy: a 1 GiB device copy (calibrates the HBM byte counters); "
                         "bkw: the 20-step RK4 BKW error curve in FP64 and FP32")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_08806_amd import inputs, pgc
    torch.cuda.set_device(0)
    if args.mode == "copy":
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB 3 times")
        return
    if args.mode == "bkw":
        bkw_curve(torch, pgc, inputs, np)
        return
    if args.mode == "profile":
        for prec in (pgc.FP64, pgc.FP32):
            plan = make_plan(pgc, prec)
            c = plan.project(inputs.bkw_f(T0, plan.interior_velocities()))
            for _ in range(2):
                plan.coeffs_to_q(c)
            torch.cuda.synchronize()
            log("profiled %s: W=%d points=%d" % ("fp64" if prec == pgc.FP64 else "fp32",
                                                 plan.info.kernel_width, plan.info.n_points))
            plan.close()
        return

    r64 = time_variant(torch, pgc, inputs, pgc.FP64, args.steps, args.warmup)
    r32 = time_variant(torch, pgc, inputs, pgc.FP32, args.fp32_steps, args.warmup)
    evals64 = 4 * args.steps / (r64["ms"] / 1e3)
    evals32 = 4 * args.fp32_steps / (r32["ms"] / 1e3)
    rel32 = float(np.linalg.norm(r32["q0"] - r64["q0"]) / np.linalg.norm(r64["q0"]))

    info = r64["info"]
    W = info.kernel_width
    flops_per_launch = 2.0 * W ** 3 * info.n_points  # spreading: W^3 multiply-adds per point
    spread_ms = r64["stages"]["spread"] / max(1, r64["calls"])
    achieved = flops_per_launch / (spread_ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["fp64"] / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK["fp64"],
                "traffic": traffic_for("gain_binned_fp64_3d_n32")}

    line = {
        "metric": METRIC,
        "value": evals64,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (closed-form 3D BKW initial data)",
        "config": {"workload": "3D BKW, N=32 modes/dim (32768 coefficients), S=5 log map, Maxwell "
                               "B=1/(4pi), 64 sphere directions (8x8 product rule), RK4 dt=0.1 from "
                               "t=6.5; step = one RK4 step (4 Q evaluations) + FP64 moments",
                   "kernel_width": W, "upsample": info.upsample, "n_points": info.n_points,
                   "n_triples": info.n_triples},
        "roofline": roofline,
        "stage_ms_per_eval_fp64": {k: v / max(1, r64["calls"]) for k, v in r64["stages"].items()},
        "variants": {
            "fp32": {"value": evals32, "unit": "evals/s", "ms_per_step": r32["ms"] / args.fp32_steps,
                     "rel_l2_vs_fp64_path": rel32, "kernel_width": r32["info"].kernel_width,
                     "stage_ms_per_eval": {k: v / max(1, r32["calls"]) for k, v in r32["stages"].items()}},
        },
        "moments_fp64_final": r64["moments"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
