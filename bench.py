"""Throughput benchmark of the IPM hot path on one MI355X.

Default line (--form headline): the batching workload -- 64 independent 2D
Euler problems with three uncertainties (sides 64/128/256, 1.59e6 cells),
per-cell total degree 1..4 (16..140 dual unknowns per cell), 5^3
Gauss-Legendre nodes, Euler entropy, Rusanov, CFL 0.5 -- stepped together
(one launch per Newton kernel shape and one update launch per step).  A step
is one IPM time step of every problem: for every cell the dual Newton solve
to tau = 1e-10, the kinetic flux at the nodes and the moment update.  The
value is the mixed-precision form (Hessian on the matrix cores in split BF16
with FP32 accumulation, stored FP32 inverse Hessians reused while they
contract, FP64 gradient, tau test and solve); beside it the plain FP64 form
and the FP64 form with stored inverses, on the same steps from the same
states.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IPM cell-updates/sec (dual Newton+flux) vs plain FP64; p50/p99 solve latency"
PEAK_FP64_VALU = 78.6e12  # MI355X vector FP64, FLOP/s
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_dual_sod8192.json")
PROFILE_TRAFFIC_HEADLINE = os.path.join(ROOT, "profiles", "traffic_chord_batch64.json")
KERNEL_SOURCES = ["dual.hpp", "device_common.hpp"]
HEADLINE_SOURCES = ["dual.hpp", "device_common.hpp", "chord.hpp", "chord_big.hpp", "dual_big.hpp"]


def kernel_hash(sources=None):
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
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


def cpu_baseline(spec, budget_s, warmup=0):
    """The oracle (plain FP64 C, OpenMP over cells) on the host cores: the
    GPU's untimed warm-up steps untimed here too, then the following steps
    of the same workload (the start of the GPU's timed window) until
    budget_s seconds of stepping."""
    import oracle
    from paper_1912_09238_amd import workloads as W
    oracle.build()
    o = oracle.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
    if warmup > 0:
        o.step(warmup)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    info = o.info
    return {"value": spec["nx"] * steps / dt, "unit": "cell-updates/s",
            "cores": oracle.load().orc_threads(), "kind": "oracle",
            "sample": "time steps %d..%d of the same Sod workload (%d cells; the GPU's timed "
                      "window starts at step %d), %.1f s" % (warmup, warmup + steps - 1, spec["nx"],
                                                             warmup, dt),
            "kbar": info["newton_iters"] / max(1, info["cell_updates"])}


MIXED = dict(precision="bf16", hessian_reuse=2)
PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s


def class_flops(n, m, Q, listed, iterations, fresh, c_closure=80, evaluations=0):
    """Algorithmic FP64-equivalent flops of a size class's Newton work
    (symmetric minimum): each solved cell evaluates the ansatz and the
    gradient once on entry; an iteration with a fresh Hessian adds the
    assembly, the Cholesky solve and the re-evaluation; an iteration with a
    stored inverse adds its matrix-vector product and the re-evaluation.
    Where the kernel counts its passes over the nodes (evaluations: entry
    and every line-search trial), those replace the one re-evaluation per
    iteration."""
    N = n // m
    f_eval = 2 * m * N * Q + Q * c_closure
    f_grad = 2 * m * N * Q + m * N
    f_hess = (m * (m + 1) // 2) * (N * (N + 1) // 2) * Q * 2
    f_chol = n ** 3 / 3 + 2 * n * n + n
    f_eg = f_eval + f_grad
    stale = iterations - fresh
    if evaluations:
        return evaluations * f_eg + fresh * (f_hess + f_chol) + stale * 2 * n * n
    return listed * f_eg + fresh * (f_hess + f_chol + f_eg) + stale * (2 * n * n + f_eg)


def class_bytes(n, m, Q, listed, iterations, fresh, variant):
    """Algorithmic HBM bytes of a size class's Newton work (each byte once,
    the Newton loop on chip): per solved cell the dual and the moments read,
    the dual and the nodal ansatz written; with stored inverses (variant
    bit 1, and the chord kernels, variant 10) the cell's n x n FP32 inverse
    read once, and written once per fresh Hessian.  Re-reads of the inverse
    by later steps of the same launch are the implementation's (served
    from L2 when the active cells' inverses fit there), not the method's."""
    b = listed * (3 * n + Q * m) * 8
    if variant & 2:
        b += (listed + fresh) * n * n * 4
    return b


def _gpu_context(**kw):
    import torch
    from paper_1912_09238_amd import binding
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.init()
    return binding.Context(device=0, stream=torch.cuda.current_stream().cuda_stream, **kw)


def batch_form(args):
    """Batching form: 64 uneven 2D Euler problems with three uncertainties,
    per-cell total degree 1..4 (4..35 modes, 16..140 unknowns), 5^3 nodes,
    stepped together (one launch per kernel shape, graph replay); the same
    batch in the mixed-precision form (BF16 MFMA Hessians and inexact-Hessian
    Newton on every cell) and in the inexact-Hessian form alone, each with its
    E/Var difference from the FP64 batch."""
    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    specs = W.batch_problems(count=args.batch_count)
    nodes, _ = binding.quadrature(3, 5)
    ids, cells, hist = [], 0, np.zeros(5, dtype=np.int64)
    t_setup = time.perf_counter()
    for k, spec in enumerate(specs):
        cd = W.cell_degrees(spec)
        hist += np.bincount(cd, minlength=5)
        ids.append(ctx.set_problem(spec, ic_nodal=W.ic_nodal(spec, nodes), cell_degree=cd))
        cells += spec["nx"] * spec["ny"]
        if k % 8 == 7:
            print("batch set-up: %d problems, %d cells" % (k + 1, cells), file=sys.stderr, flush=True)
    t_setup = time.perf_counter() - t_setup
    tuned = ctx.autotune(ids, steps_per_candidate=1) if args.autotune else 0
    ctx.step(ids, args.batch_warmup, wait=True)
    before = ctx.step(ids, 0, wait=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(ids, args.batch_steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    after = ctx.step(ids, 0, wait=True)
    assert all(a["status"] == 0 for a in after), after
    done = sum((a["steps"] - b["steps"]) * (sp["nx"] * sp["ny"])
               for a, b, sp in zip(after, before, specs))
    newton = sum(a["newton_iters"] - b["newton_iters"] for a, b in zip(after, before))
    value = done / elapsed
    def e_var(ids_):
        out = []
        for pid in ids_:
            m = ctx.moments(pid)
            out.append((m[:, :, 0].copy(), np.sum(m[:, :, 1:] ** 2, axis=2)))
        return out
    ev64 = e_var(ids)
    # the same problems stepped one at a time (per-problem launches), fewer steps
    seq_steps = max(1, args.batch_steps // 10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for pid in ids:
        ctx.step(pid, seq_steps)
    torch.cuda.synchronize()
    seq_value = cells * seq_steps / (time.perf_counter() - t1)
    for pid in ids:
        ctx.release(pid)
    # the same problems, same warm-up and timed steps from the same initial
    # states, in the mixed-precision form (BF16 MFMA Hessians, inexact-Hessian
    # Newton with FP32 inverses reused on every cell, FP64 tau test) and in the
    # inexact-Hessian form alone (FP64 Hessians)
    forms = {}
    for fname, extra, label in (
            ("mixed_precision_batch", dict(precision="bf16", hessian_reuse=2),
             "bf16 MFMA Hessian + inexact-Hessian Newton on all cells, FP64 tau"),
            ("inexact_hessian_batch", dict(hessian_reuse=2),
             "FP64 Hessian + inexact-Hessian Newton on all cells, FP64 tau")):
        pids = [ctx.set_problem(dict(spec, **extra), ic_nodal=W.ic_nodal(spec, nodes),
                                cell_degree=W.cell_degrees(spec)) for spec in specs]
        ctx.step(pids, args.batch_warmup, wait=True)
        pbefore = ctx.step(pids, 0, wait=True)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ctx.step(pids, args.batch_steps)
        torch.cuda.synchronize()
        f_elapsed = time.perf_counter() - t4
        pafter = ctx.step(pids, 0, wait=True)
        assert all(a["status"] == 0 for a in pafter), pafter
        ev = e_var(pids)
        for pid in pids:
            ctx.release(pid)
        num_e = sum(np.abs(a[0] - b[0]).sum() for a, b in zip(ev, ev64))
        den_e = sum(np.abs(b[0]).sum() for b in ev64)
        num_v = sum(np.abs(a[1] - b[1]).sum() for a, b in zip(ev, ev64))
        den_v = sum(np.abs(b[1]).sum() for b in ev64)
        f_value = done / f_elapsed
        forms[fname] = {"value": f_value, "speedup_vs_fp64": f_value / value,
                        "ms_per_step": f_elapsed / args.batch_steps * 1e3, "form": label,
                        "kbar": sum(a["newton_iters"] - b["newton_iters"]
                                    for a, b in zip(pafter, pbefore)) / max(1, done),
                        "rel_l1_vs_fp64": {"E": float(num_e / den_e), "Var": float(num_v / den_v)}}
    prec_value = forms["mixed_precision_batch"]["value"]
    print("batch form: fp64 %.4g, bf16 + reuse %.4g cell-updates/s" % (value, prec_value),
          file=sys.stderr, flush=True)
    # many small problems: 64 Burgers shocks of 512 cells, degree 5 -- here the
    # launch count, not the cell work, decides, and the batch shares launches
    small = [W.burgers_shock(nx=512, degree=5, qpd=12, t_end=0.0) for _ in range(64)]
    bn, _ = binding.quadrature(1, 12)
    sids = [ctx.set_problem(sp, ic_nodal=W.ic_nodal(sp, bn)) for sp in small]
    ctx.step(sids, 4, wait=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.step(sids, 200)
    torch.cuda.synchronize()
    small_batched = 64 * 512 * 200 / (time.perf_counter() - t2)
    t3 = time.perf_counter()
    for _ in range(20):
        for pid in sids:
            ctx.step(pid, 1)
    torch.cuda.synchronize()
    small_seq = 64 * 512 * 20 / (time.perf_counter() - t3)
    for pid in sids:
        ctx.release(pid)
    ctx.close()
    return {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.batch_steps, "warmup": args.batch_warmup,
        "ms_per_step": elapsed / args.batch_steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch%d_euler2d_p3_deg1to4_q125_fp64" % len(specs),
                   "problems": len(specs), "cells": cells,
                   "cells_by_degree": {str(k): int(hist[k]) for k in range(1, 5)},
                   "parallelism": "single-gpu"},
        "one_problem_at_a_time": {"value": seq_value, "steps": seq_steps},
        "mixed_precision_batch": forms["mixed_precision_batch"],
        "inexact_hessian_batch": forms["inexact_hessian_batch"],
        "small_problems_64x512_burgers_deg5": {"batched": small_batched,
                                                "one_problem_at_a_time": small_seq},
        "setup_s": t_setup, "autotuned_shapes": tuned,
        "kbar": newton / max(1, done),
    }


def _batch_ids(ctx, specs, nodes, extra):
    from paper_1912_09238_amd import workloads as W
    return [ctx.set_problem(dict(spec, **extra), ic_nodal=W.ic_nodal(spec, nodes),
                            cell_degree=W.cell_degrees(spec)) for spec in specs]


def _class_totals(ctx, ids):
    """Newton counters summed over problems per kernel shape."""
    tot = {}
    for pid in ids:
        for c in ctx.class_stats(pid):
            key = (c["workgroup"], c["lanes"], c["variant"])
            t = tot.setdefault(key, {"n_min": c["n_min"], "n_max": c["n_max"], "cells": 0,
                                     "listed": 0, "iterations": 0, "fresh": 0,
                                     "evaluations": 0})
            t["n_min"] = min(t["n_min"], c["n_min"])
            t["n_max"] = max(t["n_max"], c["n_max"])
            for k in ("cells", "listed", "iterations", "fresh", "evaluations"):
                t[k] += c[k]
    return tot


def _kernel_name(m, key):
    workgroup, lanes, variant = key
    if variant == 10:
        if workgroup:
            return "newton_chord_big_batched<%d,%d>" % (m, lanes // 16)
        return "newton_chord_batched<%d,%d>" % (m, lanes)
    if workgroup:
        return "newton_big_batched<%d,%d,%d>" % (m, lanes // 16, variant)
    return "newton_batched<%d,%d,%d>" % (m, lanes, variant)


def timed_batch(ctx, specs, nodes, extra, warmup, steps, m=4, Q=125):
    """Set up the batch in one form, run `warmup` untimed steps, then time
    `steps` steps launched one kernel at a time on the context's stream with
    a HIP event pair around every Newton launch.  Returns the rate, the
    per-kernel table (launches, mean device time, algorithmic flops per
    launch from the per-class Newton counters of the same window) and the
    E / Var of every problem."""
    import torch
    ids = _batch_ids(ctx, specs, nodes, extra)
    cells = sum(sp["nx"] * sp["ny"] for sp in specs)
    ctx.step(ids, warmup, wait=True)
    before = ctx.step(ids, 0, wait=True)
    c0 = _class_totals(ctx, ids)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    ctx.step(ids, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = ctx.timing(False)
    lt = ctx.launch_times()
    after = ctx.step(ids, 0, wait=True)
    c1 = _class_totals(ctx, ids)
    assert all(a["status"] == 0 for a in after), after
    assert all(a["steps"] - b["steps"] == steps for a, b in zip(after, before))
    newton = sum(a["newton_iters"] - b["newton_iters"] for a, b in zip(after, before))
    kernels = []
    for t in lt:
        key = (t["workgroup"], t["lanes"], t["variant"])
        c = c1[key]
        d = {k: c[k] - c0[key][k] for k in ("listed", "iterations", "fresh", "evaluations")}
        assert c["n_min"] == c["n_max"], ("one size per class", key, c)
        n = c["n_max"]
        flops = class_flops(n, m, Q, d["listed"], d["iterations"], d["fresh"],
                            evaluations=d["evaluations"])
        nbytes = class_bytes(n, m, Q, d["listed"], d["iterations"], d["fresh"], key[2])
        avg = t["ms"] / t["launches"] * 1e-3
        kernels.append({"kernel": _kernel_name(m, key), "unknowns": n,
                        "cells": c["cells"], "launches": t["launches"], "us_avg": avg * 1e6,
                        "share_of_step": t["ms"] * 1e-3 / elapsed,
                        "listed_per_launch": d["listed"] / t["launches"],
                        "iterations_per_listed": d["iterations"] / max(1, d["listed"]),
                        "fresh_per_listed": d["fresh"] / max(1, d["listed"]),
                        "evaluations_per_iteration":
                            d["evaluations"] / max(1, d["iterations"]) if d["evaluations"] else None,
                        "flops_per_launch": flops / t["launches"],
                        "bytes_per_launch": nbytes / t["launches"],
                        "achieved_tflops": flops / t["launches"] / avg / 1e12,
                        "achieved_gbs": nbytes / t["launches"] / avg / 1e9})
    kernels.sort(key=lambda k: -k["us_avg"] * k["launches"])
    ev = []
    for pid in ids:
        mo = ctx.moments(pid)
        ev.append((mo[:, :, 0].copy(), np.sum(mo[:, :, 1:] ** 2, axis=2)))
    for pid in ids:
        ctx.release(pid)
    return {"value": cells * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
            "kbar": newton / (cells * steps), "update_ms_per_step": tm["update_ms"] / steps,
            "kernels": kernels}, ev


def _rel_e_var(ev, ev_ref):
    out = {}
    for name, j in (("E", 0), ("Var", 1)):
        num1 = sum(np.abs(a[j] - b[j]).sum() for a, b in zip(ev, ev_ref))
        den1 = sum(np.abs(b[j]).sum() for b in ev_ref)
        num2 = sum(((a[j] - b[j]) ** 2).sum() for a, b in zip(ev, ev_ref))
        den2 = sum((b[j] ** 2).sum() for b in ev_ref)
        out[name] = {"l1": float(num1 / den1), "l2": float(np.sqrt(num2 / den2))}
    return out


def cpu_baseline_batch(specs, warmup, steps, budget_s):
    """The oracle (plain FP64 C, OpenMP over cells) on the host cores over the
    same step window as the GPU (warmup untimed steps, then `steps` timed
    steps) on the batch's problems of side 64, in order, until budget_s
    seconds of timed stepping."""
    import oracle
    from paper_1912_09238_amd import workloads as W
    oracle.build()
    done_cells, timed, used, newton, cu = 0, 0.0, [], 0, 0
    for k, spec in enumerate(specs):
        if spec["nx"] != 64:
            continue
        o = oracle.Oracle(spec, ic_fn=lambda nd, s=spec: W.ic_nodal(s, nd),
                          cell_degree=W.cell_degrees(spec))
        o.step(warmup)
        i0 = o.info
        t0 = time.perf_counter()
        o.step(steps)
        timed += time.perf_counter() - t0
        i1 = o.info
        assert i1["status"] == 0 and i1["steps"] - i0["steps"] == steps, i1
        newton += i1["newton_iters"] - i0["newton_iters"]
        cu += i1["cell_updates"] - i0["cell_updates"]
        done_cells += o.cells * steps
        used.append(k)
        del o
        if timed >= budget_s:
            break
    return {"value": done_cells / timed, "unit": "cell-updates/s",
            "cores": oracle.load().orc_threads(), "kind": "oracle",
            "sample": "problems %s of the batch (side 64, 4096 cells each), steps %d..%d "
                      "(the GPU's timed window), %.1f s, FP64 exact Newton" % (
                          used, warmup, warmup + steps - 1, timed),
            "kbar": newton / max(1, cu)}


def serving_leg(args):
    """A short window of the serving workload (Poisson arrivals at 200/s, 60 %
    Burgers / 40 % Sod, degree 3..9) through the library's serving loop, FP64
    form: p50 / p99 latency from arrival to moments on the host, offered and
    served cell-updates/s."""
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context(hbm_budget=int(args.budget_gb * 2 ** 30))
    reqs = []
    for spec in W.request_stream(rate=args.rate, duration=args.serve_window):
        nodes, _ = binding.quadrature(1, spec["quad_per_dim"])
        reqs.append({"spec": spec, "arrival": spec["arrival"], "ic_nodal": W.ic_nodal(spec, nodes)})
    res = ctx.serve(reqs, steps_per_round=args.round, max_active=args.max_active, moments=False)
    ctx.close()
    assert all(r["status"] == 0 for r in res), [r for r in res if r["status"]][:3]
    lat = np.array([r["latency"] for r in res])
    work = sum(r["steps"] * rq["spec"]["nx"] for r, rq in zip(res, reqs))
    makespan = max(r["finished"] for r in res)
    return {"workload": "serve_poisson%d_burgers60_sod40_fp64_%gs" % (int(args.rate),
                                                                       args.serve_window),
            "requests": len(reqs), "latency_s": {"p50": float(np.percentile(lat, 50)),
                                                 "p99": float(np.percentile(lat, 99))},
            "offered_cell_updates_per_s": work / args.serve_window,
            "served_cell_updates_per_s": work / makespan, "makespan_s": makespan}


def headline_form(args):
    """The default line: the 64-problem batch in the mixed-precision form
    (value), the plain FP64 form and the FP64 form with stored inverses, on
    the same window of steps; roofline of the value form's dominant Newton
    kernel; the oracle on the host over the same window; a short serving
    leg."""
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    specs = W.batch_problems(count=64)
    nodes, _ = binding.quadrature(3, 5)
    cells = sum(sp["nx"] * sp["ny"] for sp in specs)
    hist = np.zeros(5, dtype=np.int64)
    for sp in specs:
        hist += np.bincount(W.cell_degrees(sp), minlength=5)
    forms = {}
    evs = {}
    reps = {}
    for name, extra in (("mixed", MIXED), ("fp64", {}), ("fp64_reuse", dict(hessian_reuse=2))):
        # each repeat sets the batch up afresh and times the same window; the
        # line reports the repeat with the median rate
        runs = []
        for k in range(max(1, args.repeats)):
            runs.append(timed_batch(ctx, specs, nodes, extra, args.warmup, args.steps))
            print("headline %s repeat %d: %.4g cell-updates/s, %.1f ms/step" % (
                name, k, runs[-1][0]["value"], runs[-1][0]["ms_per_step"]), file=sys.stderr, flush=True)
        runs.sort(key=lambda r: r[0]["value"])
        forms[name], evs[name] = runs[len(runs) // 2]
        reps[name] = [r[0]["value"] for r in runs]
    ctx.close()
    mixed, fp64, reuse = forms["mixed"], forms["fp64"], forms["fp64_reuse"]
    dom = mixed["kernels"][0]
    # the binding roof of the dominant kernel: HBM below the FP64 ridge
    # (78.6 TFLOP/s / 8 TB/s = 9.8 flop per byte), FP64 ALU above
    ai = dom["flops_per_launch"] / max(1.0, dom["bytes_per_launch"])
    if ai < PEAK_FP64_VALU / PEAK_HBM:
        roof = {"bound": "hbm", "achieved": dom["achieved_gbs"], "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": dom["achieved_gbs"] * 1e9 / PEAK_HBM}
    else:
        roof = {"bound": "alu", "achieved": dom["achieved_tflops"],
                "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                "frac": dom["achieved_tflops"] * 1e12 / PEAK_FP64_VALU}
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC_HEADLINE):
        prof = json.load(open(PROFILE_TRAFFIC_HEADLINE))
        if prof.get("kernel_hash") == kernel_hash(HEADLINE_SOURCES) and \
                prof.get("kernel") == dom["kernel"]:
            traffic = prof.get("bytes_per_launch")
    roof.update({"traffic": traffic, "kernel": dom["kernel"], "us_avg": dom["us_avg"],
                 "flops_per_launch": dom["flops_per_launch"],
                 "bytes_per_launch": dom["bytes_per_launch"], "flop_per_byte": ai,
                 "unknowns": dom["unknowns"]})
    out = {
        "metric": METRIC, "value": mixed["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": "batch64_euler2d_p3_deg1to4_q125_mixed_precision",
                   "problems": len(specs), "cells": cells,
                   "cells_by_degree": {str(k): int(hist[k]) for k in range(1, 5)},
                   "form": "BF16-split MFMA Hessian (cells of 65..96 unknowns) + stored FP32 "
                           "inverse Hessians on every cell; FP64 gradient, tau test, solve",
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "repeats": {"count": max(1, args.repeats), "value_is": "median",
                    "mixed": reps["mixed"], "fp64": reps["fp64"], "fp64_reuse": reps["fp64_reuse"]},
        "fp64_batch": {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                       "kbar": fp64["kbar"], "kernels": fp64["kernels"]},
        "speedup_vs_fp64": mixed["value"] / fp64["value"],
        "fp64_reuse_batch": {"value": reuse["value"], "ms_per_step": reuse["ms_per_step"],
                             "speedup_vs_fp64": reuse["value"] / fp64["value"]},
        # where the speed-up comes from: the inexact-Hessian Newton (stored
        # inverses, chord kernels) alone, and the BF16 Hessian on top of it
        "attribution": {"inverse_reuse": reuse["value"] / fp64["value"],
                        "bf16_hessian": mixed["value"] / reuse["value"]},
        "bf16_share": mixed["value"] / reuse["value"],
        "mixed_rel_vs_fp64": _rel_e_var(evs["mixed"], evs["fp64"]),
        "kbar": mixed["kbar"], "kernels": mixed["kernels"],
        "update_ms_per_step": mixed["update_ms_per_step"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(specs, args.warmup, args.steps, args.cpu_seconds)
    if args.serve_window > 0:
        out["serving"] = serving_leg(args)
    if args.copy_calibration:
        _copy_calibration()
    return out


def _copy_calibration():
    """A 1 GiB device-to-device copy (three times): the reference for scaling
    the HBM counters of the profiled kernels."""
    import torch
    x = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def precision_form(args):
    """Precision form: 2D Euler bump on a periodic 512 x 512 grid, two
    uncertainties, total degree 5 (21 modes, 84 unknowns per cell), 8 x 8
    nodes, the same steps in the plain FP64 form (exact Newton), with the
    split-BF16 MFMA Hessian, and with the inexact-Hessian Newton (stored FP32
    inverse Hessians reused while they contract) in FP64 and with the BF16
    Hessian.  The tau test stays FP64 in every variant; the line reports the
    BF16 + reuse variant and the relative L1 difference of E and Var of every
    variant against the plain form."""
    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    spec = W.bump2d(n=args.prec_n, degree=5, qpd=8)
    nodes, _ = binding.quadrature(2, 8)
    ic = W.ic_nodal(spec, nodes)
    cells = spec["nx"] * spec["ny"]
    out = {}
    variants = (("fp64", {}), ("bf16", dict(precision="bf16")),
                ("fp64_reuse", dict(hessian_reuse=1)),
                ("bf16_reuse", dict(precision="bf16", hessian_reuse=1)))
    for name, kw in variants:
        pid = ctx.set_problem(dict(spec, **kw), ic_nodal=ic)
        ctx.step(pid, args.prec_warmup, wait=True)
        b = ctx.step(pid, 0, wait=True)[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(pid, args.prec_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        a = ctx.step(pid, 0, wait=True)[0]
        assert a["status"] == 0, a
        out[name] = {"value": cells * args.prec_steps / el, "ms_per_step": el / args.prec_steps * 1e3,
                     "kbar": (a["newton_iters"] - b["newton_iters"]) / (cells * args.prec_steps),
                     "moments": ctx.moments(pid)}
        ctx.release(pid)
        print("precision form: %s %.4g cell-updates/s" % (name, out[name]["value"]),
              file=sys.stderr, flush=True)
    ctx.close()
    m64 = out["fp64"]["moments"]
    rel = lambda a, b: float(np.abs(a - b).sum() / np.abs(b).sum())
    for k, v in out.items():
        m = v.pop("moments")
        v["rel_l1_vs_fp64"] = {"E": rel(m[:, :, 0], m64[:, :, 0]),
                               "Var": rel(np.sum(m[:, :, 1:] ** 2, axis=2),
                                          np.sum(m64[:, :, 1:] ** 2, axis=2))}
        v["speedup_vs_fp64"] = v["value"] / out["fp64"]["value"]
    r = out["bf16_reuse"]
    return {
        "metric": METRIC, "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.prec_steps, "warmup": args.prec_warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16-mfma-hessian+fp32-inverse-reuse/f64", "data": "synthetic",
        "config": {"workload": "euler2d_bump_%dx%d_deg5_q64" % (args.prec_n, args.prec_n),
                   "cells": cells, "n": 84, "Q": 64, "parallelism": "single-gpu"},
        "speedup_vs_fp64": r["speedup_vs_fp64"],
        "rel_l1_vs_fp64": r["rel_l1_vs_fp64"],
        "variants": out,
    }


def serve_form(args):
    """Serving form: Poisson request stream (60 % Burgers, 40 % Sod, degree
    3..9) through the library's serving loop; latency from arrival to moments
    on the host."""
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context(hbm_budget=int(args.budget_gb * 2 ** 30))
    reqs = []
    for spec in W.request_stream(rate=args.rate, duration=args.duration):
        nodes, _ = binding.quadrature(1, spec["quad_per_dim"])
        reqs.append({"spec": spec, "arrival": spec["arrival"], "ic_nodal": W.ic_nodal(spec, nodes)})
    t0 = time.perf_counter()
    res = ctx.serve(reqs, steps_per_round=args.round, max_active=args.max_active, moments=False)
    wall = time.perf_counter() - t0
    assert all(r["status"] == 0 for r in res), [r for r in res if r["status"]][:3]
    lat = np.array([r["latency"] for r in res])
    work = sum(r["steps"] * rq["spec"]["nx"] for r, rq in zip(res, reqs))
    makespan = max(r["finished"] for r in res)
    # the same 1D stream in the reduced-precision request form: BF16 Hessian
    # (which the register-row kernels of these cells, n <= 30, do not use)
    # and the inexact-Hessian Newton on every cell
    rq_m = [dict(rq, spec=dict(rq["spec"], precision="bf16", hessian_reuse=2)) for rq in reqs]
    res_m = ctx.serve(rq_m, steps_per_round=args.round, max_active=args.max_active, moments=False)
    assert all(r["status"] == 0 for r in res_m), [r for r in res_m if r["status"]][:3]
    lat_m = np.array([r["latency"] for r in res_m])
    work_m = sum(r["steps"] * rq["spec"]["nx"] for r, rq in zip(res_m, reqs))
    span_m = max(r["finished"] for r in res_m)
    one_d_mixed = {"form": "bf16 + inexact-Hessian Newton on every cell (BF16 unused at n <= 30)",
                   "served_cell_updates_per_s": work_m / span_m, "makespan_s": span_m,
                   "latency_s": {"p50": float(np.percentile(lat_m, 50)),
                                 "p99": float(np.percentile(lat_m, 99))},
                   "served_ratio_vs_fp64": (work_m / span_m) / (work / makespan)}
    print("serve form, 1D mixed: %.4g cell-updates/s, p50 %.3f s" % (
        work_m / span_m, one_d_mixed["latency_s"]["p50"]), file=sys.stderr, flush=True)
    # 2D requests (21 unknowns per variable, 84 per cell), where the precision
    # form applies: the same stream served in the FP64 form and in the
    # mixed-precision form (BF16 Hessian + inverse reuse), at an open-loop
    # rate the GPU keeps up with and at a rate that saturates it; moments of
    # each request compared between the forms
    two_d = {}
    n2, _ = binding.quadrature(2, 8)
    for rate in args.rate_2d:
        stream = W.request_stream_2d(rate=rate, duration=args.duration)
        row, moms = {}, {}
        for form, kw in (("fp64", {}), ("mixed", dict(precision="bf16", hessian_reuse=1))):
            rq2 = [{"spec": dict(sp, **kw), "arrival": sp["arrival"],
                    "ic_nodal": W.ic_nodal(sp, n2)} for sp in stream]
            r2 = ctx.serve(rq2, steps_per_round=args.round, max_active=args.max_active,
                           moments=True)
            assert all(r["status"] == 0 for r in r2), [r for r in r2 if r["status"]][:3]
            l2 = np.array([r["latency"] for r in r2])
            w2 = sum(r["steps"] * sp["nx"] * sp["ny"] for r, sp in zip(r2, stream))
            m2 = max(r["finished"] for r in r2)
            moms[form] = [r["moments"] for r in r2]
            row[form] = {"served_cell_updates_per_s": w2 / m2, "makespan_s": m2,
                         "latency_s": {"p50": float(np.percentile(l2, 50)),
                                       "p99": float(np.percentile(l2, 99))}}
            row["offered_cell_updates_per_s"] = w2 / args.duration
            print("serve form, 2D at %g/s %s: %.4g cell-updates/s, p50 %.4f s, p99 %.4f s" % (
                rate, form, w2 / m2, row[form]["latency_s"]["p50"],
                row[form]["latency_s"]["p99"]), file=sys.stderr, flush=True)
        pairs = list(zip(moms["mixed"], moms["fp64"]))
        num_e = sum(np.abs(a[:, :, 0] - b[:, :, 0]).sum() for a, b in pairs)
        den_e = sum(np.abs(b[:, :, 0]).sum() for _, b in pairs)
        num_v = sum(np.abs((a[:, :, 1:] ** 2).sum(2) - (b[:, :, 1:] ** 2).sum(2)).sum()
                    for a, b in pairs)
        den_v = sum((b[:, :, 1:] ** 2).sum() for _, b in pairs)
        row["requests"] = len(stream)
        row["mixed_rel_l1_vs_fp64"] = {"E": float(num_e / den_e), "Var": float(num_v / den_v)}
        row["speedup_served"] = (row["mixed"]["served_cell_updates_per_s"] /
                                 row["fp64"]["served_cell_updates_per_s"])
        row["p50_ratio_fp64_over_mixed"] = (row["fp64"]["latency_s"]["p50"] /
                                            row["mixed"]["latency_s"]["p50"])
        row["p99_ratio_fp64_over_mixed"] = (row["fp64"]["latency_s"]["p99"] /
                                            row["mixed"]["latency_s"]["p99"])
        two_d["poisson%g" % rate] = row
    ctx.close()
    return {
        "metric": METRIC, "value": work / makespan, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serve_poisson%d_burgers60_sod40_fp64" % int(args.rate),
                   "requests": len(reqs), "arrival_window_s": args.duration,
                   "steps_per_round": args.round, "max_active": args.max_active,
                   "hbm_budget_gb": args.budget_gb, "parallelism": "single-gpu"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "offered_cell_updates_per_s": work / args.duration,
        "served_cell_updates_per_s": work / makespan, "makespan_s": makespan, "wall_s": wall,
        "requests_1d_mixed": one_d_mixed,
        "requests_2d_fp64_vs_mixed": two_d,
    }


def adapt_form(args):
    """Adaptive form (Sec. 5, Alg. ad-IPM): levels (total degrees) move every
    step by the smoothness indicator of the density, one level at a time.
    Main line: the 2D Euler bump on a periodic 512 x 512 grid, two
    uncertainties, levels 1..5 (3..21 modes, 12..84 unknowns per cell),
    8 x 8 nodes, thresholds 1e-5 / 1e-4 (those of the paper's 2D study),
    against the fixed degree 5 over the same steps; relative L1 difference of
    E and Var of every conserved variable.  Also: whole Sod trajectories
    (8192 cells, levels 2..9, thresholds 2e-5 / 2e-4) against degree 9."""
    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    rel = lambda a, b: float(np.abs(a - b).sum() / np.abs(b).sum())
    # ---- 2D bump: fixed steps
    base = W.bump2d(n=args.prec_n, degree=5, qpd=8, p=2)
    spec = dict(base, adapt=1, min_degree=1, delta_lo=1e-5, delta_hi=1e-4)
    nodes, _ = binding.quadrature(2, 8)
    ic = W.ic_nodal(base, nodes)
    cells = base["nx"] * base["ny"]
    res = {}
    # the adaptive run also with inverse reuse (BF16 Hessian): the
    # precision form on top of the adaptivity
    spec_r = dict(spec, hessian_reuse=1, precision="bf16")
    for name, sp in (("fixed", base), ("adaptive", spec), ("adaptive_reuse", spec_r)):
        pid = ctx.set_problem(sp, ic_nodal=ic)
        ctx.step(pid, args.prec_warmup, wait=True)
        b = ctx.step(pid, 0, wait=True)[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(pid, args.prec_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        a = ctx.step(pid, 0, wait=True)[0]
        assert a["status"] == 0, a
        dg = ctx.degrees(pid)
        res[name] = {"value": cells * args.prec_steps / el, "ms_per_step": el / args.prec_steps * 1e3,
                     "kbar": (a["newton_iters"] - b["newton_iters"]) / (cells * args.prec_steps),
                     "moments": ctx.moments(pid), "levels": np.bincount(dg, minlength=6),
                     "degrees": dg}
        ctx.release(pid)
        print("adaptive form, 2D: %s %.4g cell-updates/s" % (name, res[name]["value"]),
              file=sys.stderr, flush=True)
    mf, ma = res["fixed"]["moments"], res["adaptive"]["moments"]
    lv = res["adaptive"]["levels"]
    n_of = np.array([(d + 1) * (d + 2) // 2 for d in range(6)]) * 4
    # ---- Sod: whole trajectories
    sbase = W.sod()
    sspec = dict(sbase, adapt=1, min_degree=2, delta_lo=2e-5, delta_hi=2e-4)
    snodes, _ = binding.quadrature(1, sbase["quad_per_dim"])
    sic = W.ic_nodal(sbase, snodes)
    warm = ctx.set_problem(sspec, ic_nodal=sic)
    ctx.step(warm, 50, wait=True)
    ctx.release(warm)
    sod = {}
    for name, sp in (("fixed", sbase), ("adaptive", sspec)):
        pid = ctx.set_problem(sp, ic_nodal=sic)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            ctx.step(pid, 1024)
            info = ctx.query(pid)
            if info["done"]:
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert info["status"] == 0, info
        sod[name] = {"seconds": el, "steps": info["steps"], "moments": ctx.moments(pid),
                     "value": sbase["nx"] * info["steps"] / el}
        ctx.release(pid)
    ctx.close()
    sf, sa = sod["fixed"]["moments"], sod["adaptive"]["moments"]
    out = {
        "metric": METRIC, "value": res["adaptive"]["value"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.prec_steps, "warmup": args.prec_warmup,
        "ms_per_step": res["adaptive"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "euler2d_bump_%dx%d_adaptive_deg1to5_q64_fp64" % (
                       args.prec_n, args.prec_n),
                   "cells": cells, "delta_lo": 1e-5, "delta_hi": 1e-4, "levels": [1, 5],
                   "parallelism": "single-gpu"},
        "fixed_degree5": {"value": res["fixed"]["value"], "ms_per_step": res["fixed"]["ms_per_step"],
                          "kbar": res["fixed"]["kbar"]},
        "speedup_vs_fixed": res["adaptive"]["value"] / res["fixed"]["value"],
        "adaptive_with_bf16_inverse_reuse": {
            "value": res["adaptive_reuse"]["value"],
            "ms_per_step": res["adaptive_reuse"]["ms_per_step"],
            "kbar": res["adaptive_reuse"]["kbar"],
            "speedup_vs_fixed": res["adaptive_reuse"]["value"] / res["fixed"]["value"],
            "rel_l1_vs_adaptive": {
                "E": rel(res["adaptive_reuse"]["moments"][:, :, 0], ma[:, :, 0]),
                "Var": rel(np.sum(res["adaptive_reuse"]["moments"][:, :, 1:] ** 2, axis=2),
                           np.sum(ma[:, :, 1:] ** 2, axis=2))},
            "cells_with_other_level": int(np.sum(res["adaptive_reuse"]["degrees"] !=
                                                  res["adaptive"]["degrees"]))},
        "kbar": res["adaptive"]["kbar"],
        "final_levels": {str(k): int(v) for k, v in enumerate(lv) if v},
        "mean_unknowns_per_cell": float((lv * n_of).sum() / lv.sum()),
        "rel_l1_vs_fixed": {v: {"E": rel(ma[:, k, 0], mf[:, k, 0]),
                                "Var": rel(np.sum(ma[:, k, 1:] ** 2, axis=1),
                                           np.sum(mf[:, k, 1:] ** 2, axis=1))}
                            for k, v in enumerate(("rho", "rho_u", "rho_v", "E"))},
        "sod_trajectory": {
            "workload": "sod1d_nx8192_adaptive_deg2to9_q20 vs degree 9, t_end 0.14",
            "adaptive": {"seconds": sod["adaptive"]["seconds"], "steps": sod["adaptive"]["steps"],
                         "value": sod["adaptive"]["value"]},
            "fixed": {"seconds": sod["fixed"]["seconds"], "steps": sod["fixed"]["steps"],
                      "value": sod["fixed"]["value"]},
            "rel_l1_vs_fixed": {"E_rho": rel(sa[:, 0, 0], sf[:, 0, 0]),
                                "Var_rho": rel(np.sum(sa[:, 0, 1:] ** 2, axis=1),
                                               np.sum(sf[:, 0, 1:] ** 2, axis=1))}},
    }
    if not args.no_cpu:
        import oracle
        oracle.build()
        o = oracle.Oracle(spec, ic_fn=lambda nd: W.ic_nodal(spec, nd))
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            o.step(1)
            k += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cells * k / dt, "unit": "cell-updates/s",
                               "cores": oracle.load().orc_threads(), "kind": "oracle",
                               "sample": "first %d adaptive time steps of the same 2D workload, "
                                         "%.1f s" % (k, dt)}
    return out


def steady_form(args):
    """Steady form (Sec. 4 and 5): the steady inflow problem (Burgers,
    log-barrier entropy, Dirichlet inflow 1 + 0.2 xi, closed-form steady state
    uhat = (1, 0.2/sqrt(3), 0, ...)) on 2048 cells at degree 9, 10 nodes,
    iterated to the steady residual 1e-10 by IPM (Alg. IPM), one-shot IPM
    (Alg. osIPM), adaptive one-shot (Alg. adosIPM, levels 1..9) and adaptive
    one-shot with refinement retardation (level cap 1 until the residual
    reaches 3e-3); time to the steady state and distance to the closed form."""
    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    base = W.steady_inflow(nx=args.steady_nx, degree=9, qpd=10, eps=1e-10)
    nodes, _ = binding.quadrature(1, 10)
    ic, dn = W.ic_nodal(base, nodes), W.dirichlet_nodal(base, nodes)
    ad = dict(adapt=1, min_degree=1, delta_lo=1e-6, delta_hi=5e-2)
    variants = [("IPM", dict(base)), ("osIPM", dict(base, one_shot=1)),
                ("adosIPM", dict(base, one_shot=1, **ad)),
                ("readosIPM", dict(base, one_shot=1, retard=((1, 3e-3), (9, 0.0)), **ad))]
    want = np.zeros(10)
    want[0], want[1] = 1.0, 0.2 / np.sqrt(3.0)
    warm = ctx.set_problem(variants[3][1], ic_nodal=ic, dirichlet=dn)
    ctx.step(warm, 20, wait=True)
    ctx.release(warm)
    res = {}
    for name, sp in variants:
        pid = ctx.set_problem(sp, ic_nodal=ic, dirichlet=dn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            ctx.step(pid, 512)
            info = ctx.query(pid)
            if info["done"] or info["steps"] >= 200000:
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert info["status"] == 0 and info["done"], (name, info)
        mom = ctx.moments(pid)
        lv = np.bincount(ctx.degrees(pid), minlength=10)
        ctx.release(pid)
        res[name] = {"seconds": el, "steps": info["steps"], "newton_iters": info["newton_iters"],
                     "value": base["nx"] * info["steps"] / el,
                     "max_err_vs_closed_form": float(np.max(np.abs(mom[:, 0, :] - want))),
                     "final_levels": {str(k): int(v) for k, v in enumerate(lv) if v}}
        print("steady form: %s %d steps %.3f s" % (name, info["steps"], el), file=sys.stderr,
              flush=True)
    ctx.close()
    r = res["readosIPM"]
    return {
        "metric": METRIC, "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": r["steps"], "warmup": 20, "ms_per_step": r["seconds"] / r["steps"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "steady_inflow_burgers_nx%d_deg9_q10_logbarrier_fp64" % args.steady_nx,
                   "cells": args.steady_nx, "steady_eps": 1e-10, "parallelism": "single-gpu"},
        "time_to_steady_s": {k: v["seconds"] for k, v in res.items()},
        "speedup_vs_IPM": {k: res["IPM"]["seconds"] / v["seconds"] for k, v in res.items()},
        "variants": res,
    }


def sg_form(args):
    """Stochastic-Galerkin baseline (App. A): Burgers' equation with an
    uncertain shock (8192 cells, degree 9, N = 10) stepped as IPM with the
    log-barrier entropy, as SG (quadratic entropy) with the kinetic
    Lax-Friedrichs flux on 14 nodes (exact for SG), and as SG with the
    analytic triple-product flux; time per step of each."""
    import torch
    from paper_1912_09238_amd import binding
    from paper_1912_09238_amd import workloads as W
    ctx = _gpu_context()
    nx, steps = 8192, args.sg_steps
    base = W.burgers_shock(nx=nx, degree=9, qpd=14, t_end=0.0)
    sg = dict(base, entropy="quadratic")
    variants = [("IPM_log_barrier", base), ("SG_kinetic_LF", sg),
                ("SG_analytic_flux", dict(sg, flux="sg_analytic"))]
    nodes, _ = binding.quadrature(1, 14)
    res = {}
    for name, sp in variants:
        pid = ctx.set_problem(sp, ic_nodal=W.ic_nodal(sp, nodes))
        ctx.step(pid, 10, wait=True)
        b = ctx.query(pid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(pid, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        a = ctx.query(pid)
        assert a["status"] == 0, (name, a)
        ctx.timing(True)
        ctx.step(pid, 50)
        tm = ctx.timing(False)
        ctx.release(pid)
        res[name] = {"value": nx * steps / el, "ms_per_step": el / steps * 1e3,
                     "dual_us_per_step": tm["dual_ms"] / 50 * 1e3,
                     "update_us_per_step": tm["update_ms"] / 50 * 1e3,
                     "kbar": (a["newton_iters"] - b["newton_iters"]) / (nx * steps)}
        print("sg form: %s %.4f ms per step" % (name, res[name]["ms_per_step"]), file=sys.stderr,
              flush=True)
    ctx.close()
    r = res["SG_analytic_flux"]
    return {
        "metric": METRIC, "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": 10, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "burgers_shock_nx%d_deg9_sg_baseline" % nx, "cells": nx, "N": 10,
                   "Q": 14, "parallelism": "single-gpu"},
        "variants": res,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--form", choices=["headline", "plain", "batch", "serve", "precision",
                                       "adapt", "steady", "sg"],
                    default="headline",
                    help="headline: the 64-problem batch, mixed precision vs FP64 (default); "
                         "plain: the Sod tube in FP64; batch / serve / precision / adapt / "
                         "steady / sg: the batching, serving, precision, adaptive, steady "
                         "(one-shot, retardation) and stochastic-Galerkin studies")
    ap.add_argument("--serve-window", type=float, default=0.25,
                    help="headline: seconds of request arrivals in the serving leg (0: none)")
    ap.add_argument("--steady-nx", type=int, default=2048)
    ap.add_argument("--sg-steps", type=int, default=400)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--rate-2d", type=float, nargs="+", default=[40.0, 400.0])
    ap.add_argument("--duration", type=float, default=1.0)
    ap.add_argument("--round", type=int, default=8)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--prec-n", type=int, default=512)
    ap.add_argument("--prec-steps", type=int, default=20)
    ap.add_argument("--prec-warmup", type=int, default=2)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (headline 20, plain 5000)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before them (headline 5, plain 20)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--repeats", type=int, default=3,
                    help="headline: repeats of each form's timed window (median reported)")
    ap.add_argument("--trajectory-steps", type=int, default=0,
                    help="steps of one full trajectory if known (skips probing it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (cells would shard "
              "spatially with a one-cell halo per step)", file=sys.stderr)
        sys.exit(2)
    if args.form == "headline":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 5 if args.warmup is None else args.warmup
        print(json.dumps(headline_form(args)), flush=True)
        return
    if args.form == "batch":
        # --steps / --warmup, when given, are the batch form's timed and
        # untimed steps (else --batch-steps / --batch-warmup)
        args.batch_steps = args.batch_steps if args.steps is None else args.steps
        args.batch_warmup = args.batch_warmup if args.warmup is None else args.warmup
    args.steps = 5000 if args.steps is None else args.steps
    args.warmup = 20 if args.warmup is None else args.warmup
    if args.form == "batch":
        print(json.dumps(batch_form(args)), flush=True)
        return
    if args.form == "serve":
        print(json.dumps(serve_form(args)), flush=True)
        return
    if args.form == "precision":
        print(json.dumps(precision_form(args)), flush=True)
        return
    if args.form == "adapt":
        print(json.dumps(adapt_form(args)), flush=True)
        return
    if args.form == "steady":
        print(json.dumps(steady_form(args)), flush=True)
        return
    if args.form == "sg":
        print(json.dumps(sg_form(args)), flush=True)
        return

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
                     "kernel": "newton_kernel<3,32,4>", "dual_us_avg": dual_avg_s * 1e6,
                     "update_us_avg": upd_avg_s * 1e6,
                     "flops_per_launch": flops_per_launch},
        "kbar": newton / cell_updates,
        "max_newton_iters": maxit,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds, args.warmup)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
