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


def time_steps(pfk, torch, A, B, method, b, steps, warmup, mmax=NU, graph_iters=10, **opts):
    """Steady-state timing of a CG/CR-type method: the window is filled first
    (at least mmax + 2 iterations), then exactly `steps` iterations are timed
    between two device synchronisations.  Returns the open session and seconds."""
    x = torch.zeros_like(b)
    S = pfk.Session(A, B, method, b, x, rtol=0.0, maxit=10 ** 7, mmax=mmax, graph_iters=graph_iters, **opts)
    S.start()
    S.iterate(max(warmup, mmax + 2))
    info0 = S.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info1 = S.sync()
    if info1.status not in (0, 1) or info1.iterations - info0.iterations != steps:
        raise RuntimeError(f"{method}: expected {steps} steady iterations, got "
                           f"{info1.iterations - info0.iterations} (status {info1.status_name})")
    return S, dt


def time_cycles(pfk, torch, A, B, method, b, cycles, m, **opts):
    """Restarted GMRES types: one warm-up cycle, then `cycles` timed cycles of
    m iterations, each followed by the restart's start-up (new residual,
    basis vector and pipeline fill) as a restarted solve does.  Returns seconds."""
    x = torch.zeros_like(b)
    S = pfk.Session(A, B, method, b, x, rtol=0.0, maxit=10 ** 7, mmax=m, graph_iters=m, **opts)
    S.start()
    S.iterate(m)
    S.start()
    S.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(cycles):
        S.iterate(m)
        S.start()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.iterate(m)
    info = S.sync()
    S.close()
    if info.iterations != m:
        raise RuntimeError(f"{method}: a cycle ran {info.iterations} iterations, expected {m}")
    return dt


def time_to_solution(pfk, torch, A, B, method, b, rtol, maxit, mmax, **opts):
    """One full solve from x = 0 (graphs captured inside the timed call)."""
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = pfk.solve(A, B, method, b, x, rtol=rtol, maxit=maxit, mmax=mmax, graph_iters=10, **opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"seconds": round(dt, 4), "iterations": info.iterations, "restarts": info.restarts,
            "converged": bool(info.converged), "true_rel_resid": info.true_rel_resid,
            "solves_per_s": round(1.0 / dt, 4)}, x


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
    steady-state mean of `kernel`: its dispatches after the first `skip` (the
    window fills during the first nu iterations of a solve, so the early
    dispatches move fewer bytes; the profiled command runs one such solve)."""
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
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the FP64 PIPEFCG/FCG pair (for profiler runs)")
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

    def rate(method, Bx, **opts):
        S, dt = time_steps(pfk, torch, A, Bx, method, b, args.steps, args.warmup, **opts)
        return S, {"it_per_s": round(args.steps / dt, 3), "ms_per_step": round(dt / args.steps * 1e3, 4)}

    results, sessions = {}, {}
    for method in ("pipefcg", "fcg"):
        log(f"timing {method}: {args.warmup} warm-up + {args.steps} steps")
        sessions[method], results[method] = rate(method, B)
        log(f"{method}: {results[method]['it_per_s']:.1f} it/s")

    main_m = args.method
    other = "fcg" if main_m == "pipefcg" else "pipefcg"
    # per-kernel event timing of the dominant kernel, on its own stream
    log("kernel timing pass")
    prof = sessions[main_m].profile(args.profile_iters)
    upd_name = "k_pipefcg_update" if main_m == "pipefcg" else "k_multidot"
    ms, launches = prof.get(upd_name, (float("nan"), 0))
    avg_ms = ms / max(launches, 1)
    upd_bytes = window_update_bytes(main_m, NU, N) if main_m == "pipefcg" else (NU + 3) * 8.0 * N
    achieved = upd_bytes / (avg_ms * 1e-3) / 1e9
    kernels = {k: {"avg_ms": round(v[0] / max(v[1], 1), 4), "launches": v[1]} for k, v in prof.items()}
    for S in sessions.values():
        S.close()
    sessions.clear()

    it_bytes = {m: iteration_bytes(m, NU, INNER, N) for m in ("pipefcg", "fcg")}
    eff = {m: it_bytes[m] * results[m]["it_per_s"] / 1e9 for m in results}

    extra = {}
    if not args.headline_only:
        # unpipelined baseline with a blocking (host-synchronised) reduction
        log("timing fcg host-sync")
        S, extra["fcg_host_sync"] = rate("fcg", B, host_sync=1)
        S.close()
        # mixed precision: FP32 inner sweeps on BF16 viscosity, FP64 outer
        Bm = pfk.Precond(A, "jacobi_pcg", INNER, precision=pfk.FP32_BF16COEF)
        for method in ("pipefcg", "fcg"):
            log(f"timing {method} mixed")
            S, extra[f"{method}_mixed"] = rate(method, Bm)
            S.close()
        # block-Jacobi inner solve (8^3 blocks, 5 PCG steps each), FP64 and mixed
        Bb = pfk.Precond(A, "block_jacobi_pcg", INNER, block=8)
        Bbm = pfk.Precond(A, "block_jacobi_pcg", INNER, precision=pfk.FP32_BF16COEF, block=8)
        for tag, Bx in (("block", Bb), ("block_mixed", Bbm)):
            for method in ("pipefcg", "fcg"):
                log(f"timing {method} {tag}")
                S, extra[f"{method}_{tag}"] = rate(method, Bx)
                S.close()
        del Bm, Bb, Bbm
        # time to solution at rtol 1e-8 on config 2 (128^3, same recipe): the 256^3
        # sinker needs more than a few thousand iterations with these inner solves.
        # The global inner CG makes PIPEFCG stagnate, so solves use the block form;
        # the mixed solution's error against the FP64 one is stated.
        log("generating the 128^3 sinker workload (config 2)")
        p2 = gen.config_problem("cfg2", seed=0)
        A2 = pfk.Operator(p2.dim, p2.n, p2.eta)
        b2 = torch.as_tensor(p2.b).cuda()
        tts = {"workload": "128^3 sinker (20 spheres, eta 1e4/1), nu_max 30, block-Jacobi PCG (8^3, 5 steps)"}
        xs = {}
        for tag, prec in (("block", pfk.FP64), ("block_mixed", pfk.FP32_BF16COEF)):
            Bx = pfk.Precond(A2, "block_jacobi_pcg", INNER, precision=prec, block=8)
            for method in ("pipefcg", "fcg"):
                log(f"solving {method} {tag} (128^3) to rtol 1e-8")
                tts[f"{method}_{tag}"], xs[(method, tag)] = time_to_solution(
                    pfk, torch, A2, Bx, method, b2, 1e-8, 8000, NU)
        for method in ("pipefcg", "fcg"):
            x64, xm = xs[(method, "block")], xs[(method, "block_mixed")]
            tts[f"{method}_block_mixed"]["rel_err_vs_fp64_solution"] = float(
                torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64))
        extra["time_to_solution_rtol1e-8"] = tts
        del xs, A2, b2, p2

        # config 3: 256^3 convection-diffusion, GMRES(5) inner solve in FP32 on BF16 viscosity
        log("generating the 256^3 convection-diffusion workload")
        p3 = gen.config_problem("cfg3", seed=0)
        A3 = pfk.Operator(p3.dim, p3.n, p3.eta, p3.vel)
        B3 = pfk.Precond(A3, "jacobi_gmres", INNER, precision=pfk.FP32_BF16COEF)
        b3 = torch.as_tensor(p3.b).cuda()
        del p3
        sigma = pfk.estimate_sigma(A3, B3)
        cycles = max(1, math.ceil(args.steps / NU))
        conv = {"workload": "256^3 conv-diff sinker (cell Peclet 5), outer FP64, B = GMRES(5) FP32/BF16",
                "sigma": sigma}
        for method in ("pipefgmres", "fgmres"):
            log(f"timing {method}: {cycles} cycles of {NU}")
            opts = {"shift_sigma": sigma} if method == "pipefgmres" else {}
            dt = time_cycles(pfk, torch, A3, B3, method, b3, cycles, NU, **opts)
            conv[method] = {"it_per_s": round(cycles * NU / dt, 3), "ms_per_step": round(dt / (cycles * NU) * 1e3, 4)}
        for method in ("pipegcr", "gcr"):
            log(f"timing {method}")
            S, dt = time_steps(pfk, torch, A3, B3, method, b3, args.steps, args.warmup)
            S.close()
            conv[method] = {"it_per_s": round(args.steps / dt, 3), "ms_per_step": round(dt / args.steps * 1e3, 4)}
        extra["conv_diff_256"] = conv
        del A3, B3, b3

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 thread; about a minute)")
        cpu = cpu_baseline(prob, main_m)

    value = results[main_m]["it_per_s"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "outer_iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[main_m]["ms_per_step"],
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
            other: results[other],
            "pipelined_over_unpipelined": round(results["pipefcg"]["it_per_s"] / results["fcg"]["it_per_s"], 4),
            "algorithmic_GBps_whole_iteration": {m: round(v, 1) for m, v in eff.items()},
            "algorithmic_bytes_per_iteration": it_bytes,
            **extra,
        },
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
