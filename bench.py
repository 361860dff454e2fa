#!/usr/bin/env python3
"""Throughput of the pipelined flexible Krylov hot path on one MI355X.

A step is one outer iteration of the solver over the 256^3 variable-viscosity
sinker system (20 spheres at viscosity 1e4 in a unit cube, Dirichlet, FP64,
window nu_max = 30, preconditioner = 5 iterations of Jacobi-PCG from zero):
the fused window update with its single reduction, the reduction's finish and
scalar recurrences on a second stream, the inner solve and the operator
apply.  The solve runs with rtol = 0 so every timed step is a steady-state
iteration; the inputs are resident in HBM before timing starts.

Prints ONE JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "outer iters/s & HBM GB/s 256^3 PIPEFCG vs FCG; solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0
NU = 30
INNER = 5


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def window_update_bytes(method: str, nu: int, N: int) -> float:
    """Algorithmic HBM bytes of one launch of the method's fused window update.

    PIPEFCG (k_pipefcg_update): reads the four windows (4 nu vectors) plus
    u, w, m, n, r, x and writes p, s, q, z, x, r, u, w: (4 nu + 14) * 8 B per
    unknown.  FCG's window work is split over two kernels (dots: nu + 2 reads
    and 1 write; maxpy: nu + 1 reads, 1 write)."""
    if method == "pipefcg":
        return (4 * nu + 14) * 8.0 * N
    return (2 * nu + 5) * 8.0 * N


def iteration_bytes(method: str, nu: int, k: int, N: int) -> float:
    """Algorithmic HBM bytes per steady-state outer iteration (FP64 vectors,
    eta read once per operator apply, D^-1 stored).  Inner Jacobi-PCG with k
    steps: A_1 reads v-inputs and D^-1 and writes p, q; each B_j reads p, q,
    rho (or the v-inputs), y, D^-1 and writes y, rho; each A_j (j>1) reads
    rho, D^-1, p and writes p, q; every stencil pass also reads eta."""
    W = 8.0
    pc = (2 + 1 + 1 + 2)            # A_1: two v inputs, D^-1, eta; writes p, q
    pc += (k - 1) * (5 + 2)         # B_j: reads p, q, rho|v(2), y(j>1), D^-1 ~ 5; writes 2
    pc += (k - 1) * (4 + 2)         # A_j: rho, D^-1, p, eta; writes p, q
    if method == "pipefcg":
        upd = 4 * nu + 14
        tail = 5 + 2                # m = u + y + alpha p_k (+eta), n = A m: reads u, y, p, eta; writes m, n
        return (upd + pc + tail) * W * N
    fcg = (2 * nu + 5)              # dots + maxpy
    fcg += 4 + 2                    # x, r update: reads x, p, r, s; writes x, r
    fcg += 3 + 1                    # u = y + alpha p_k with dots (reads y, p, r): 3 + window counted above
    fcg += 2 + 1                    # s = A p: reads p, eta; writes s
    return (fcg + pc - 1) * W * N


def time_steps(pfk, torch, A, B, method, b, steps, warmup, graph_iters=10):
    x = torch.zeros_like(b)
    S = pfk.Session(A, B, method, b, x, rtol=0.0, maxit=10 ** 7, mmax=NU, graph_iters=graph_iters)
    S.start()
    S.iterate(max(warmup, NU + 2))       # fill the window: steady state
    info0 = S.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.iterate(steps)
    torch.cuda.synchronize()
    info1 = S.sync()
    dt = time.perf_counter() - t0
    if info1.status not in (0, 1) or info1.iterations - info0.iterations != steps:
        raise RuntimeError(f"{method}: expected {steps} steady iterations, got "
                           f"{info1.iterations - info0.iterations} (status {info1.status_name})")
    return S, dt


def cpu_baseline(prob, method):
    """The FP64 oracle on the host: one outer iteration of the same workload,
    timed as (start-up + 1 iteration) minus (start-up alone), one thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    A = oracle.StencilOperator(prob.dim, prob.n, prob.eta)
    with threadpool_limits(1):
        B = oracle.make_pc("jacobi_pcg", A, INNER)
        t = time.perf_counter()
        oracle.solve(method, A, B, prob.b, rtol=0.0, maxit=0, nu_max=NU)
        t_start = time.perf_counter() - t
        t = time.perf_counter()
        oracle.solve(method, A, B, prob.b, rtol=0.0, maxit=1, nu_max=NU)
        t_one = time.perf_counter() - t
    per_it = max(t_one - t_start, 1e-9)
    return {"value": 1.0 / per_it, "unit": "outer_iters/s", "cores": 1, "kind": "oracle",
            "sample": f"256^3 {method.upper()} workload: start-up + 1 outer iteration ({t_one:.1f} s) minus "
                      f"start-up alone ({t_start:.1f} s), numpy FP64, 1 thread"}


def _short_kernel_name(name: str) -> str:
    base = name.split("(")[0].replace("void ", "").strip()
    head, sep, tmpl = base.partition("<")
    return head.split("::")[-1] + (("<" + tmpl.replace("pfk::", "")) if sep else "")


def trace_summary(trace_csv: str, kernel: str, skip: int) -> str:
    """Per-kernel statistics from a rocprofv3 kernel trace (CSV), plus the
    steady-state mean of `kernel`: its dispatches after the first `skip` of
    every run of consecutive dispatches (the window fills during the first nu
    iterations, so early dispatches move fewer bytes)."""
    import csv
    rows = []
    with open(trace_csv, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), _short_kernel_name(r["Kernel_Name"]),
                         int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    stats = {}
    for _, name, ns in rows:
        s = stats.setdefault(name, [0, 0])
        s[0] += 1
        s[1] += ns
    lines = [f"{'kernel':48s} {'calls':>7s} {'avg_ms':>10s} {'total_ms':>10s}"]
    for name, (c, tot) in sorted(stats.items(), key=lambda kv: -kv[1][1])[:20]:
        lines.append(f"{name[:48]:48s} {c:7d} {tot / c / 1e6:10.4f} {tot / 1e6:10.2f}")
    durs = [ns for _, name, ns in rows if name == kernel]
    steady = durs[skip:]
    if steady:
        steady_sorted = sorted(steady)
        lines.append(f"\n{kernel}: {len(durs)} dispatches; steady state (dispatch {skip + 1} on): "
                     f"{len(steady)} dispatches, mean {sum(steady) / len(steady) / 1e6:.4f} ms, "
                     f"median {steady_sorted[len(steady) // 2] / 1e6:.4f} ms, "
                     f"min {steady_sorted[0] / 1e6:.4f} ms, max {steady_sorted[-1] / 1e6:.4f} ms")
    return "\n".join(lines)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--trace-summary":
        sp = argparse.ArgumentParser()
        sp.add_argument("--trace-summary", required=True, help="rocprofv3 *_kernel_trace.csv")
        sp.add_argument("--kernel", default="k_pipefcg_update")
        sp.add_argument("--skip", type=int, default=NU + 1)
        a = sp.parse_args()
        print(trace_summary(a.trace_summary, a.kernel, a.skip))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--method", default="pipefcg", choices=["pipefcg", "fcg"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("multi-GPU runs are not part of this build (one GPU per box); use --gpus 1")
        sys.exit(2)

    import torch
    import gen
    import paper_1511_07226_amd as pfk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("generating the 256^3 sinker workload")
    prob = gen.config_problem("cfgM", seed=0)
    N = prob.N
    A = pfk.Operator(prob.dim, prob.n, prob.eta)
    B = pfk.Precond(A, "jacobi_pcg", INNER)
    b = torch.as_tensor(prob.b).cuda()

    results = {}
    sessions = {}
    for method in ("pipefcg", "fcg"):
        log(f"timing {method}: {args.warmup} warm-up + {args.steps} steps")
        S, dt = time_steps(pfk, torch, A, B, method, b, args.steps, args.warmup)
        results[method] = {"it_per_s": args.steps / dt, "ms_per_step": dt / args.steps * 1e3}
        sessions[method] = S
        log(f"{method}: {results[method]['it_per_s']:.1f} it/s")

    main_m = args.method
    other = "fcg" if main_m == "pipefcg" else "pipefcg"
    # per-kernel event timing of the dominant kernel, on its own stream
    log("kernel timing pass")
    prof = sessions[main_m].profile(args.profile_iters)
    upd_name = "k_pipefcg_update" if main_m == "pipefcg" else "k_fcg_dots"
    ms, launches = prof.get(upd_name, (float("nan"), 0))
    avg_ms = ms / max(launches, 1)
    upd_bytes = window_update_bytes(main_m, NU, N) if main_m == "pipefcg" else (NU + 3) * 8.0 * N
    achieved = upd_bytes / (avg_ms * 1e-3) / 1e9
    kernels = {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in prof.items()}
    for S in sessions.values():
        S.close()

    it_bytes = {m: iteration_bytes(m, NU, INNER, N) for m in ("pipefcg", "fcg")}
    eff = {m: it_bytes[m] * results[m]["it_per_s"] / 1e9 for m in results}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 thread; about a minute)")
        cpu = cpu_baseline(prob, main_m)

    value = results[main_m]["it_per_s"]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "outer_iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(results[main_m]["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{main_m.upper()} 256^3 variable-viscosity sinker (20 spheres, eta 1e4/1), "
                               f"7-point FP64, nu_max={NU}, B = {INNER}-step Jacobi-PCG (global), rtol=0 steady state",
                   "unknowns": N, "method": main_m, "nu_max": NU, "inner_its": INNER},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": upd_name, "avg_ms": round(avg_ms, 4),
                     "algorithmic_bytes_per_launch": upd_bytes},
        "cpu_baseline": cpu,
        "compare": {
            other: {"it_per_s": round(results[other]["it_per_s"], 3),
                    "ms_per_step": round(results[other]["ms_per_step"], 4)},
            "pipelined_over_unpipelined": round(results["pipefcg"]["it_per_s"] / results["fcg"]["it_per_s"], 4),
            "algorithmic_GBps_whole_iteration": {m: round(v, 1) for m, v in eff.items()},
            "algorithmic_bytes_per_iteration": it_bytes,
        },
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
