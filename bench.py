"""Throughput benchmark of the IPM hot path on one MI355X.

A step is one IPM time step of the whole workload: for every cell the dual
Newton solve to tau = 1e-10, the kinetic Rusanov flux at the quadrature
nodes and the moment update (plus the device-side time step).  Workload:
1D Euler Sod tube, 8192 cells, Legendre degree 9 (N = 10, 30 dual unknowns
per cell), 20 Gauss-Legendre nodes, Euler entropy, CFL 0.5, t_end = 0.14,
FP64 throughout.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IPM cell-updates/sec (dual Newton+flux) vs plain FP64; p50/p99 solve latency"
PEAK_FP64_VALU = 78.6e12  # MI355X vector FP64, FLOP/s
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_dual_sod8192.json")
KERNEL_SOURCES = ["dual.hpp", "device_common.hpp"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1912_09238_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def flops_per_cell(m, N, Q, c_closure=80):
    """Algorithmic FP64 flops of the dual solve (symmetric minimum):
    per Newton iteration and for the final gradient + tau test."""
    n = m * N
    f_eval = 2 * m * N * Q + Q * c_closure
    f_grad = 2 * m * N * Q + m * N
    f_hess = (m * (m + 1) // 2) * (N * (N + 1) // 2) * Q * 2
    f_chol = n ** 3 / 3 + 2 * n * n + n
    return f_eval + f_grad + f_hess + f_chol, f_eval + f_grad


def cpu_baseline(spec, budget_s):
    """The oracle (plain FP64 C, OpenMP over cells) on the host cores: the
    first steps of the same workload until budget_s seconds of stepping."""
    import oracle
    from paper_1912_09238_amd import workloads as W
    oracle.build()
    o = oracle.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    info = o.info
    return {"value": spec["nx"] * steps / dt, "unit": "cell-updates/s",
            "cores": oracle.load().orc_threads(), "kind": "oracle",
            "sample": "first %d time steps of the same Sod workload (%d cells), %.1f s" % (
                steps, spec["nx"], dt),
            "kbar": info["newton_iters"] / max(1, info["cell_updates"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--trajectory-steps", type=int, default=0,
                    help="steps of one full trajectory if known (skips probing it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = binding.Context(device=0, stream=stream.cuda_stream)
    spec = W.sod()
    nodes, _ = binding.quadrature(spec["p"], spec["quad_per_dim"])
    ic = W.ic_nodal(spec, nodes)
    m, N, Q = 3, 10, 20
    cells = spec["nx"]

    # trajectory length (untimed; also warms the kernels)
    if args.trajectory_steps > 0:
        L = args.trajectory_steps
    else:
        pid = ctx.set_problem(spec, ic_nodal=ic)
        while True:
            ctx.step(pid, 512)
            traj = ctx.query(pid)
            if traj["done"]:
                break
        L = traj["steps"]
        assert traj["status"] == 0 and traj["done"], traj
        ctx.release(pid)

    def fresh_instances(total):
        k = max(1, -(-total // L))
        return [ctx.set_problem(spec, ic_nodal=ic) for _ in range(k)]

    def split_plan(ids, warm, count):
        """(warmup chunks, timed chunks): warm + count steps spread over
        instances of trajectory length L, in order."""
        chunks, left, inst, used = [], warm + count, 0, 0
        while left > 0:
            take = min(left, L - used)
            chunks.append((ids[inst], take))
            left -= take
            used += take
            if used == L:
                inst, used = inst + 1, 0
        warm_plan, timed_plan, acc = [], [], 0
        for pid_, n_ in chunks:
            w = min(n_, max(0, warm - acc))
            if w:
                warm_plan.append((pid_, w))
            if n_ - w:
                timed_plan.append((pid_, n_ - w))
            acc += n_
        return warm_plan, timed_plan

    # ---- timed pass (no instrumentation)
    ids = fresh_instances(args.warmup + args.steps)
    warm_plan, timed_plan = split_plan(ids, args.warmup, args.steps)
    for pid_, n_ in warm_plan:
        ctx.step(pid_, n_)
    before = {i: ctx.query(i) for i in ids}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pid_, n_ in timed_plan:
        ctx.step(pid_, n_)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    after = {i: ctx.query(i) for i in ids}
    steps_done = sum(after[i]["steps"] - before[i]["steps"] for i in ids)
    newton = sum(after[i]["newton_iters"] - before[i]["newton_iters"] for i in ids)
    maxit = max(after[i]["max_iters"] for i in ids)
    assert all(after[i]["status"] == 0 for i in ids), after
    assert steps_done == args.steps, (steps_done, args.steps)
    for i in ids:
        ctx.release(i)
    cell_updates = cells * args.steps
    value = cell_updates / elapsed

    # ---- instrumented repeat of the same steps: per-launch HIP events on the
    # context stream give the dual kernel's average duration
    ids = fresh_instances(args.warmup + args.steps)
    warm_plan, timed_plan = split_plan(ids, args.warmup, args.steps)
    for pid_, n_ in warm_plan:
        ctx.step(pid_, n_)
    ctx.timing(True)
    for pid_, n_ in timed_plan:
        ctx.step(pid_, n_)
    tm = ctx.timing(False)
    for i in ids:
        ctx.release(i)
    launches = tm["launches"]
    dual_avg_s = tm["dual_ms"] / max(1, launches) * 1e-3
    upd_avg_s = tm["update_ms"] / max(1, launches) * 1e-3
    f_it, f_fin = flops_per_cell(m, N, Q)
    flops_per_launch = (newton * f_it + cell_updates * f_fin) / args.steps
    achieved = flops_per_launch / dual_avg_s
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        prof = json.load(open(PROFILE_TRAFFIC))
        if prof.get("kernel_hash") == kernel_hash():
            traffic = prof.get("bytes_per_launch")

    if args.copy_calibration:
        x = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sod1d_nx8192_deg9_q20_euler_rusanov_fp64", "cells": cells,
                   "m": m, "N": N, "Q": Q, "tau": 1e-10, "trajectory_steps": L,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
                     "kernel": "newton_kernel<3,32>", "dual_us_avg": dual_avg_s * 1e6,
                     "update_us_avg": upd_avg_s * 1e6,
                     "flops_per_launch": flops_per_launch},
        "kbar": newton / cell_updates,
        "max_newton_iters": maxit,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
