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

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "outer iters/s & HBM GB/s 256^3 PIPEFCG vs FCG; solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0
NU = 30
INNER = 5


# HBM traffic of one steady-state k_pipefcg_update launch (256^3, nu = 30,
# autotuned geometry): the per-dispatch means over the last 7 dispatches of
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB), each scaled by what the same counter reads for a 2 GiB
# device-to-device copy (FETCH_SIZE reads 1,048,588 KiB for 2,097,152 KiB
# moved: x2.000; WRITE_SIZE reads 2,097,152: x1.000).  Valid only for the
# kernel source it was measured on (digest of its device body, of the
# load/store helpers and of the wave reduction it uses).
UPDATE_TRAFFIC = {"body_sha1": "b68eb769c76b8849", "fetch_kib": 8257680.5, "fetch_scale": 2.0,
                  "write_kib": 1052892.6, "write_scale": 1.0}


def update_traffic_digest():
    """Digest of k_pipefcg_update's device body, its load/store helpers and the
    wave reduction it calls."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1511_07226_amd", "csrc", "pfk_cg.hpp")).read()
    i = src.index("__device__ __forceinline__ double2 ld2(")
    j = src.index("k_pipefcg_update(", i)
    dev = open(os.path.join(ROOT, "paper_1511_07226_amd", "csrc", "pfk_device.hpp")).read()
    k = dev.index("template <int CTRL, int RM>")
    m = dev.index("__device__ __forceinline__ void block_partials", k)
    return hashlib.sha1((src[i:j] + dev[k:m]).encode()).hexdigest()[:16]


def update_traffic_bytes():
    """Measured bytes per launch of k_pipefcg_update, or None when its source
    has changed since the counters were taken."""
    if update_traffic_digest() != UPDATE_TRAFFIC["body_sha1"]:
        return None
    t = UPDATE_TRAFFIC
    return round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0)


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


def iteration_bytes(method: str, nu: int, k: int, N: int, pc: str = "global", mixed: bool = False) -> float:
    """Algorithmic HBM bytes per steady-state outer iteration (outer vectors
    FP64, eta read once per operator apply, D^-1 stored).  The inner solve's
    vectors and D^-1 take w bytes (8, or 4 in the mixed form) and its
    viscosity c bytes (8, or 2 for BF16).
    Global Jacobi-PCG with k steps: A_1 reads the v inputs, D^-1 and eta and
    writes p, q; each B_j reads q, rho (the v inputs for j = 1) and D^-1 and
    writes rho, and the last one (j = k - 1) also reads p_1 .. p_{k-1} and
    writes the iterate y; each A_j (j > 1) reads rho, D^-1, p and eta and
    writes p, q.  Block-Jacobi PCG: one pass reads the v inputs and eta and
    writes y.  The consumer forms m = u + B(v) (PIPEFCG) and applies A.""" 
    W = 8.0
    w, c = (4.0, 2.0) if mixed else (8.0, 8.0)
    if pc == "block":
        pcb = 2 * W + c + w                            # v inputs, eta; writes y
        tail_pc = w                                    # the consumer reads y
    else:
        pcb = 2 * W + w + c + 2 * w                    # A_1
        if k > 1:
            # B_j: reads rho (the two FP64 v inputs for j = 1), q, D^-1; writes rho
            pcb += 2 * W + 3 * w + (k - 2) * 4 * w
            pcb += (k - 1) * w + w                     # the last B: p_1 .. p_{k-1} in, y out
        pcb += (k - 1) * (3 * w + c + 2 * w)           # A_j: rho, D^-1, p, eta; writes p, q
        tail_pc = 2 * w if k > 1 else w                # the consumer reads y and p_k
    if method == "pipefcg":
        upd = (4 * nu + 14) * W
        tail = tail_pc + 2 * W + 2 * W                 # reads u, eta; writes m, n
        return (upd + pcb + tail) * N
    fcg = (2 * nu + 5) * W                             # dots + maxpy
    fcg += 6 * W                                       # x, r update: reads x, p, r, s; writes x, r
    fcg += tail_pc + 2 * W                             # u = B(r) with the dots: reads r; writes u
    fcg += 3 * W                                       # s = A p: reads p, eta; writes s
    return (fcg + pcb - W) * N                         # FCG's inner input is r alone


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


def time_to_solution(pfk, torch, A, B, method, b, rtol, maxit, mmax, repeats=5, **opts):
    """Full solves from x = 0 (graphs captured inside each timed call): the
    first solve on its own, then the median of the remaining `repeats - 1`."""
    times = []
    for _ in range(repeats):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = pfk.solve(A, B, method, b, x, rtol=rtol, maxit=maxit, mmax=mmax, graph_iters=10, **opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times[1:])) if repeats > 1 else times[0]
    return {"seconds": round(dt, 4), "first_solve_seconds": round(times[0], 4), "solves_timed": repeats,
            "iterations": info.iterations, "restarts": info.restarts,
            "converged": bool(info.converged), "true_rel_resid": info.true_rel_resid,
            "solves_per_s": round(1.0 / dt, 4)}, x


def persistent_rate(pfk, torch, A, B, method, b, steps, warmup):
    """Steady-state iterations/s of one system run by the persistent batched
    form (one cooperative launch per step, grid barriers between phases)."""
    T = pfk.Batch(method, mmax=NU, capacity=1, persistent=1)
    x = torch.zeros_like(b)
    T.add(A, B, b, x, rtol=0.0, maxit=warmup + steps + 50)
    T.step(warmup)
    T.poll()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, running = T.poll()
    T.close()
    if running != 1:
        raise RuntimeError(f"persistent {method}: the system stopped during timing")
    return steps / dt


def conv_diff_bench(pfk, torch, steps, warmup):
    """Configuration 3: 256^3 convection-diffusion sinker, outer FP64, inner
    GMRES(5) in FP32 on BF16 viscosity.  The GMRES types are timed over whole
    restart cycles (each followed by its restart's start-up), the CR types
    over steady-state iterations."""
    import gen
    log("generating the 256^3 convection-diffusion workload")
    p3 = gen.config_problem("cfg3", seed=0)
    A3 = pfk.Operator(p3.dim, p3.n, p3.eta, p3.vel)
    B3 = pfk.Precond(A3, "jacobi_gmres", INNER, precision=pfk.FP32_BF16COEF)
    b3 = torch.as_tensor(p3.b).cuda()
    del p3
    sigma = pfk.estimate_sigma(A3, B3)
    cycles = max(1, math.ceil(steps / NU))
    conv = {"workload": "256^3 conv-diff sinker (cell Peclet 5), outer FP64, B = GMRES(5) FP32/BF16",
            "sigma": sigma}
    for method in ("pipefgmres", "fgmres"):
        log(f"timing {method}: {cycles} cycles of {NU}")
        opts = {"shift_sigma": sigma} if method == "pipefgmres" else {}
        dt = time_cycles(pfk, torch, A3, B3, method, b3, cycles, NU, **opts)
        conv[method] = {"it_per_s": round(cycles * NU / dt, 3), "ms_per_step": round(dt / (cycles * NU) * 1e3, 4)}
    for method in ("pipegcr", "pipegcr_w", "gcr"):
        log(f"timing {method}")
        S, dt = time_steps(pfk, torch, A3, B3, method, b3, steps, warmup)
        S.close()
        conv[method] = {"it_per_s": round(steps / dt, 3), "ms_per_step": round(dt / steps * 1e3, 4)}
    return conv


def conv_diff_tts(pfk, torch, contrasts=(4.0, 2.0), restarts=(30, 60), maxit=3000):
    """Configuration 3 as a solve: the 256^3 convection-diffusion sinker to
    rtol 1e-8 from x = 0 by FGMRES, PIPEFGMRES, GCR and PIPEGCR (GMRES(5)
    inner solve in FP32 on BF16 viscosity), restart/window 30 and 60, at the
    configured viscosity contrast 1e4 and at 1e2; CR types with stagnation
    restarts (window 200).  Reports iterations, restarts, the true relative
    residual reached and seconds (one solve each, graphs captured inside)."""
    import gen
    out = {"workload": "256^3 conv-diff sinker (cell Peclet 5), rtol 1e-8, maxit %d, B = GMRES(5) FP32/BF16" % maxit}
    for c in contrasts:
        log(f"generating the 256^3 convection-diffusion workload, contrast 1e{c:g}")
        p = gen.make_problem(3, 256, 20, c, 0, convection=True)
        A = pfk.Operator(p.dim, p.n, p.eta, p.vel)
        B = pfk.Precond(A, "jacobi_gmres", INNER, precision=pfk.FP32_BF16COEF)
        b = torch.as_tensor(p.b).cuda()
        del p
        sigma = pfk.estimate_sigma(A, B)
        row = {}
        for method in ("fgmres", "pipefgmres", "gcr", "pipegcr"):
            for m in restarts:
                opts = {"shift_sigma": sigma} if method == "pipefgmres" else {}
                if method in ("gcr", "pipegcr"):
                    opts.update(stall_window=200, max_restarts=1000)
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = pfk.solve(A, B, method, b, x, rtol=1e-8, maxit=maxit, mmax=m, graph_iters=10, **opts)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                row[f"{method}_{m}"] = {"iterations": info.iterations, "restarts": info.restarts,
                                        "converged": bool(info.converged),
                                        "true_rel_resid": float(f"{info.true_rel_resid:.3e}"),
                                        "seconds": round(dt, 2)}
                log(f"contrast 1e{c:g} {method}({m}): {row[f'{method}_{m}']}")
        out[f"contrast_1e{c:g}"] = row
        del A, B, b
    return out


def size_sweep(pfk, torch, steps=40):
    """PIPEFCG against FCG per outer iteration on single systems of growing size
    (block-Jacobi inner solve, FP64, nu_max 30), in the graph-launched form and
    in the persistent form (grid barriers instead of kernel boundaries): where
    the one device-side reduction per iteration matters more than the
    pipelined method's extra window traffic."""
    import gen
    out = {}
    for dim, n in ((2, 64), (3, 16), (3, 32), (3, 64), (3, 128)):
        p = gen.make_problem(dim, n, 8 if dim == 2 else 20, 3.0 if dim == 2 else 4.0, seed=0)
        A = pfk.Operator(dim, n, p.eta)
        B = pfk.Precond(A, "block_jacobi_pcg", INNER, block=8)
        b = torch.as_tensor(p.b).cuda()
        row = {}
        for method in ("pipefcg", "fcg"):
            S, dt = time_steps(pfk, torch, A, B, method, b, steps, NU + 2)
            S.close()
            row[method] = round(steps / dt, 1)
            row[method + "_persistent"] = round(persistent_rate(pfk, torch, A, B, method, b, steps, NU + 2), 1)
        row["pipelined_over_unpipelined"] = round(row["pipefcg"] / row["fcg"], 3)
        row["pipelined_over_unpipelined_persistent"] = round(row["pipefcg_persistent"] / row["fcg_persistent"], 3)
        out[f"{dim}d_n{n}"] = row
    return out


def least_padding_tile(n):
    """The stencil tile width (64: 64 x 8 tiles, 32: 32 x 16) that pads an n x n
    plane least (64 on a tie)."""
    pad = {tx: -(-n // tx) * tx * -(-n // (512 // tx)) * (512 // tx) for tx in (64, 32)}
    return 64 if pad[64] <= pad[32] else 32


def batch_member_tiling(A, n, tile_x, vector_blocks, zc):
    """A batch member's launch geometry: stencil tiles of width tile_x, the
    z-range cut into chunks of about zc planes, vector_blocks workgroups for
    the vector kernels.  A single solve of a small grid wants many short
    z-marches to fill the GPU; in a batch the members together fill it, so
    each member's marches can be as long as on a large grid."""
    ty = 2 * 256 // tile_x
    tiles = -(-n // tile_x) * -(-n // ty)
    A.set_tiling(tile_x, tiles * -(-n // zc), vector_blocks)


def batched_bench(pfk, torch, steps, warmup, count=64, solve=True, batch_zc=0):
    """Configuration 4: 64 uneven SPD systems (edge 32..96, contrast 1e2..1e4),
    PIPEFCG nu_max 20 with the block-Jacobi inner solve (4 steps, FP32 on BF16
    viscosity), advanced by shared launches.  Tiling per size from the
    autotuner.  Reports steady-state batch iterations/s (every system advances
    one iteration), the same for FCG and for the systems stepped one at a time,
    and the time to solve all of them to rtol 1e-8.  batch_zc > 0 gives the
    batch member tilings of the least-padding tile width, the autotuned
    vector workgroups and z-marches of about batch_zc planes (the
    one-at-a-time comparison keeps the autotuned single-solve tilings)."""
    import gen
    NU4, K4 = 20, 4
    # the configuration gives no iteration limit: 20000 lets the slowest
    # members (contrast near 1e4 at 64^3..96^3, where PIPEFCG's recurred
    # residual stalls near 1e-7 with FP32 inner sweeps until a residual-gap
    # restart) reach the tolerance
    MAXIT4 = 20000
    STALL4 = 200        # stagnation restarts, as for serving
    probs = gen.batched_problems(count, seed=0)
    mem = []
    for p in probs:
        A = pfk.Operator(3, p.n, p.eta)
        B = pfk.Precond(A, "block_jacobi_pcg", K4, precision=pfk.FP32_BF16COEF, block=8)
        mem.append((p, A, B))
    tuning = {}
    for p, A, B in mem:
        if p.n not in tuning:
            tuning[p.n] = A.autotune(B, "pipefcg", mmax=NU4, reps=5)
    def single_tiling():
        for p, A, B in mem:
            t = tuning[p.n]
            A.set_tiling(t["tile_x"], t["stencil_target"], t["vector_blocks"])

    def batch_tiling(zc):
        for p, A, B in mem:
            batch_member_tiling(A, p.n, least_padding_tile(p.n), tuning[p.n]["vector_blocks"], zc)

    total_n = sum(A.N for _, A, _ in mem)
    bs = [torch.as_tensor(p.b).cuda() for p, _, _ in mem]
    out = {"workload": f"{count} SPD sinker systems, edge in {{32,48,64,80,96}}, {total_n} unknowns; "
                       f"nu_max {NU4}, block-Jacobi PCG ({K4} steps, FP32/BF16), outer FP64",
           "sizes": {str(n): sum(1 for p, _, _ in mem if p.n == n) for n in sorted(tuning)},
           "autotuned": {str(n): {k: v for k, v in t.items()} for n, t in tuning.items()}}

    def steady(method, persistent=0):
        T = pfk.Batch(method, mmax=NU4, capacity=count, graph_iters=10, persistent=persistent)
        xs = [torch.zeros_like(b) for b in bs]
        for (p, A, B), b, x in zip(mem, bs, xs):
            T.add(A, B, b, x, rtol=0.0, maxit=warmup + steps + 50)
        T.step(max(warmup, NU4 + 2))
        T.poll()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, running = T.poll()
        T.close()
        if running != count:
            raise RuntimeError(f"batched {method}: {count - running} systems stopped during timing")
        return steps / dt

    # optional: member tilings with the least-padding tile width and z-chunks
    # of batch_zc planes (longer z-marches than the single-solve tilings of
    # these small grids)
    if batch_zc > 0:
        batch_tiling(batch_zc)
        out["batch_zc"] = batch_zc
    else:
        single_tiling()
    for method in ("pipefcg", "fcg"):
        log(f"batched {method}: timing {steps} steps")
        r = steady(method)
        out[f"{method}_batch_iters_per_s"] = round(r, 2)
        out[f"{method}_unknown_iters_per_s"] = round(r * total_n, 1)
    # the persistent form: each step one cooperative launch, phases separated
    # by grid barriers instead of kernel boundaries
    for method in ("pipefcg", "fcg"):
        log(f"batched {method}, persistent form: timing {steps} steps")
        out[f"{method}_persistent_batch_iters_per_s"] = round(steady(method, persistent=1), 2)
    # the same systems stepped one session at a time (one per size, scaled by
    # count), with the single-solve tilings; the batch tiling is restored after
    single_tiling()
    seq_ms = 0.0
    for n in sorted(tuning):
        p, A, B = next(m for m in mem if m[0].n == n)
        S, dt = time_steps(pfk, torch, A, B, "pipefcg", torch.as_tensor(p.b).cuda(), steps, warmup, mmax=NU4)
        S.close()
        seq_ms += dt / steps * 1e3 * out["sizes"][str(n)]
    out["pipefcg_one_at_a_time_iters_per_s"] = round(1e3 / seq_ms, 2)
    out["batching_speedup"] = round(out["pipefcg_batch_iters_per_s"] * seq_ms / 1e3, 3)
    # bytes of one batched PIPEFCG iteration: window update (4 nu + 14 vectors), the
    # block solve (v in: 2 vectors, BF16 eta 2 B, FP32 y out 4 B), m, n (u, FP32 y,
    # FP64 eta in; m, n out)
    per_unknown = (4 * NU4 + 14) * 8 + (2 * 8 + 2 + 4) + (8 + 4 + 8 + 2 * 8)
    out["algorithmic_GBps_pipefcg"] = round(per_unknown * total_n * out["pipefcg_batch_iters_per_s"] / 1e9, 1)
    out["algorithmic_bytes_per_unknown_iteration"] = per_unknown
    if batch_zc > 0:
        batch_tiling(batch_zc)
    if not solve:
        return out
    log("batched pipefcg: solving all systems to rtol 1e-8")
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    code, infos = pfk.solve_batched([A for _, A, _ in mem], [B for _, _, B in mem], "pipefcg", bs, xs,
                                    rtol=1e-8, maxit=MAXIT4, mmax=NU4, graph_iters=10, stall_window=STALL4,
                                    max_restarts=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = [i.iterations for i in infos]
    nconv = sum(1 for i in infos if i.converged)
    log("batched pipefcg, persistent form: solving all systems to rtol 1e-8")
    xp = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infp = pfk.solve_batched([A for _, A, _ in mem], [B for _, _, B in mem], "pipefcg", bs, xp,
                                rtol=1e-8, maxit=MAXIT4, mmax=NU4, graph_iters=10, persistent=1,
                                stall_window=STALL4, max_restarts=100)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    out["time_to_solution_persistent"] = {"seconds": round(dtp, 3),
                                          "converged": sum(1 for i in infp if i.converged),
                                          "same_iterations_as_phased": all(a.iterations == b.iterations
                                                                           for a, b in zip(infos, infp))}
    out["time_to_solution"] = {"seconds": round(dt, 3), "converged_solves_per_s": round(nconv / dt, 2),
                               "converged": nconv,
                               "iterations_min_median_max": [min(its), sorted(its)[len(its) // 2], max(its)],
                               "max_true_rel_resid": max(i.true_rel_resid for i in infos)}
    return out


def serving_bench(pfk, torch, nreq=240, seed=0, loads=(0.9,), direct=False, per_batch=64, zc=0):
    """Configuration 5: Poisson arrivals of PIPEFCG / PIPEFGMRES requests (50/50)
    on 3D sinker grids, edge lognormal (median 40, sigma_ln 0.5) clipped to
    16..128, contrast 10^U(1,4), rtol 1e-6 or 1e-8, admitted by a memory
    budget into continuously refilled batches.  PIPEFGMRES requests use the
    5-step right-Jacobi GMRES inner solve, PIPEFCG requests the block-Jacobi
    PCG (4 steps; the global 4-step CG makes PIPEFCG stagnate), both in FP32
    on BF16 viscosity.  The capacity is measured with every request arriving
    at once; Poisson streams then offer a fraction of it.  Latency =
    completion seen by the serving loop minus arrival; rates count converged
    requests."""
    import gen
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(nreq):
        n = int(np.clip(round(float(rng.lognormal(math.log(40.0), 0.5))), 16, 128))
        method = "pipefcg" if rng.random() < 0.5 else "pipefgmres"
        rtol = 1e-6 if rng.random() < 0.5 else 1e-8
        p = gen.make_problem(3, n, 20, (1.0, 4.0), seed=10000 + i)
        A = pfk.Operator(3, n, p.eta)
        if zc > 0:
            # batch member tiling: z-marches of about zc planes, the tile width
            # that pads the grid least, the operator's vector workgroups
            batch_member_tiling(A, n, least_padding_tile(n), A.tiling()[2], zc)
        if method == "pipefgmres":
            B = pfk.Precond(A, "jacobi_gmres", 5, precision=pfk.FP32_BF16COEF)
        else:
            B = pfk.Precond(A, "block_jacobi_pcg", 4, precision=pfk.FP32_BF16COEF, block=8)
        reqs.append(dict(A=A, B=B, b=torch.as_tensor(p.b).cuda(), method=method, rtol=rtol, n=n))
    budget = 48 << 30
    MAXIT = 10000
    # window / restart length (the configuration leaves it open): 60.  With 30,
    # high-contrast requests stall -- PIPEFGMRES(30) as FGMRES(30) does, and
    # PIPEFCG with the FP32 inner sweeps and a full 30-direction window -- while
    # 60 converges them (measured per request against 10, 20, 40, 50)
    NU_SERVE = 60
    # stagnation restarts (window 200): PIPEFCG with the FP32 inner sweeps can
    # stall at a floor that scales with ||A|| ||B|| on high-contrast requests
    # (section 2.2.1's noise effect, the noise being FP32 rounding); a restart
    # from the current x rebuilds the recurrences there
    STALL = 200

    def run(arrivals):
        srv = pfk.Server(hbm_budget=budget, max_active=per_batch, step_iters=8, mmax=NU_SERVE, launch_direct=direct,
                         stall_window=STALL, max_restarts=100)
        xs = [torch.zeros_like(r["b"]) for r in reqs]
        ids, lat, conv = {}, [], 0
        by_method, failed = {}, []
        t0 = time.perf_counter()
        k, done = 0, 0
        while done < len(reqs):
            now = time.perf_counter() - t0
            while k < len(reqs) and arrivals[k] <= now:
                r = reqs[k]
                ids[srv.submit(r["A"], r["B"], r["method"], r["b"], xs[k], rtol=r["rtol"], maxit=MAXIT)] = k
                k += 1
            st = srv.stats()
            if st["active"] == 0 and st["queued"] == 0:
                if k < len(reqs):
                    time.sleep(max(0.0, min(0.002, arrivals[k] - now)))
                continue
            fin = srv.progress()
            t = time.perf_counter() - t0
            for rid in fin:
                lat.append(t - arrivals[ids[rid]])
                info = srv.result(rid)
                conv += int(info.converged)
                r = reqs[ids[rid]]
                key = f"{r['method']}_rtol{r['rtol']:.0e}"
                bym = by_method.setdefault(key, [0, 0])
                bym[0] += 1
                bym[1] += int(info.converged)
                if not info.converged and len(failed) < 12:
                    failed.append({"n": r["n"], "method": r["method"], "rtol": r["rtol"],
                                   "iterations": info.iterations, "status": info.status_name,
                                   "true_rel": float(f"{info.true_rel_resid:.3e}")})
                done += 1
                if done % 250 == 0:
                    log(f"serving: {done} of {len(reqs)} requests done at {t:.1f} s")
        total = time.perf_counter() - t0
        srv.close()
        lat = np.sort(np.array(lat))
        return {"requests": len(reqs), "seconds": round(total, 3),
                "converged_solves_per_s": round(conv / total, 2), "served_per_s": round(len(reqs) / total, 2),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2), "converged": conv,
                "served_converged_by_kind": by_method, "not_converged_sample": failed}

    log(f"serving: {nreq} requests arriving at once (capacity)")
    cap = run(np.zeros(nreq))
    out = {"workload": f"{nreq} requests, edge lognormal(40, 0.5) in 16..128, PIPEFCG/PIPEFGMRES 50/50, "
                       f"rtol 1e-6/1e-8, window/restart {NU_SERVE}, maxit {MAXIT}, stagnation restarts (window "
                       f"{STALL}); PIPEFGMRES: GMRES(5), PIPEFCG: "
                       f"block-Jacobi PCG (4), FP32/BF16 inner; budget 48 GiB, {per_batch} per batch" +
                       (", direct launches" if direct else ", graphs"),
           "edge_median": int(np.median([r["n"] for r in reqs])), "burst": cap, "poisson": {}}
    for f in loads:
        rate = f * cap["converged_solves_per_s"]
        arr = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / rate, size=nreq))
        log(f"serving: Poisson arrivals at {rate:.1f}/s ({f} x capacity)")
        out["poisson"][f"{f}x"] = {"offered_per_s": round(rate, 2), **run(arr)}
    return out


def stagnation_study(pfk, torch):
    """Section 2.2.1 (Figure 1) at scale: FCG, PIPEFCG and naive PIPEFCG
    (Alg. 7) with the seeded noisy preconditioner B(r) = r + eta ||r|| g/||g||
    on the unit-scaled Dirichlet Laplacian (eta = h^2, the stencil's 1/h^2
    cancelled so that the spectrum is of order one as in the toy), b = A x*.
    Each method runs as a full solve (true-residual check, breakdown
    restarts) to rtol 1e-10 or maxit, and reports its relative error
    ||x - x*|| / ||x*||.  Naive PIPEFCG also reports its error along one
    cycle (up to its first breakdown) at iterations 5, 10, ..., 50, then
    every 50.  Both truncation rules at 128^3; the standard one at 256^3 for
    eta = 1e-2."""
    import gen
    out = {"workload": "unit-scaled 7-point Laplacian, b = A x* (x* ~ N(0,1)), noisy B (seed 1), nu_max 30, "
                       "rtol 1e-10"}
    marks = list(range(5, 50, 5)) + list(range(50, 2001, 50))
    plan = ((128, (1e-1, 1e-2, 1e-3), (0, 1), 1000), (256, (1e-2,), (0,), 1500))
    for n, etas, truncs, maxit in plan:
        p = gen.study_problem(3, n, seed=0)
        A = pfk.Operator(3, n, p.eta)
        xs = torch.as_tensor(p.meta["x_star"]).cuda()
        b = A.apply(xs)
        xn = float(torch.linalg.vector_norm(xs))
        del p

        def rel_err(x):
            return float(f"{float(torch.linalg.vector_norm(x - xs)) / xn:.3g}")

        for trunc in truncs:
            for eta in etas:
                for method in ("fcg", "pipefcg", "pipefcg_naive"):
                    key = f"{n}^3/{'notay' if trunc else 'standard'}/eta={eta:g}/{method}"
                    B = pfk.Precond(A, "noisy", eta=eta, seed=1)
                    x = torch.zeros_like(b)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    info = pfk.solve(A, B, method, b, x, rtol=1e-10, maxit=maxit, mmax=NU, truncation=trunc,
                                     graph_iters=10)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    r = {"iterations": info.iterations, "restarts": info.restarts, "converged": info.converged,
                         "status": info.status_name, "rel_error": rel_err(x),
                         "true_rel_resid": float(f"{info.true_rel_resid:.3g}"),
                         "ms_per_iteration": round(dt / max(info.iterations, 1) * 1e3, 4)}
                    if method == "pipefcg_naive":
                        r["plateau_over_eta"] = round(r["rel_error"] / eta, 3)
                        # the error along one cycle, sampled
                        x.zero_()
                        S = pfk.Session(A, pfk.Precond(A, "noisy", eta=eta, seed=1), method, b, x, rtol=1e-10,
                                        maxit=maxit, mmax=NU, truncation=trunc, graph_iters=10)
                        S.start()
                        curve, it = [], 0
                        for stop in marks:
                            if stop > maxit:
                                break
                            S.iterate(stop - it)
                            reached = S.sync().iterations
                            curve.append([reached, rel_err(x)])
                            if reached < stop:
                                break
                            it = reached
                        S.close()
                        r["cycle_rel_error_at"] = curve
                    out[key] = r
                    log(f"stagnation {key}: {info.iterations} its, {info.restarts} restarts, "
                        f"rel error {r['rel_error']:.3g}")
        del A, xs, b
        torch.cuda.empty_cache()
    return out


def cpu_baseline(method, n=128, steady=6):
    """The FP64 oracle on the host, at steady state: the same recipe as the
    256^3 workload (20 spheres, eta 1e4/1, nu_max 30, global 5-step
    Jacobi-PCG) at n = 128 (config 2's size), which the oracle fills and times
    in 20-100 s depending on the host (at 256^3 the fill alone would take
    several minutes).  One solve runs nu_max + 1 + 2 steady iterations; each iteration
    applies B once, so the times between successive B calls are outer
    iterations.  Iterations [nu, nu + steady) run on one thread, the next
    `steady` on every host core (threadpoolctl; numpy's elementwise and
    slicing work stays on one core either way, only its BLAS dots spread).
    The rate is reported per n^3 iteration and scaled by n^3 / 256^3 to the
    256^3 unit (every step of an iteration is linear in N)."""
    import oracle
    import gen
    from threadpoolctl import threadpool_limits
    p = gen.config_problem("cfgM", seed=0, n=n)
    A = oracle.StencilOperator(p.dim, p.n, p.eta)
    Bpc = oracle.make_pc("jacobi_pcg", A, INNER)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    # B call c belongs to iteration c - 1 for PIPEFCG (its start-up applies B
    # twice) and to iteration c for FCG: start timing at iteration nu + 1
    first = NU + 2 if method == "pipefcg" else NU + 1
    stamps = []
    lim = {}

    def B(v):
        c = len(stamps)
        if c == first:
            lim["one"] = threadpool_limits(1)
        elif c == first + steady:
            lim["one"].restore_original_limits()
            lim["all"] = threadpool_limits(cores)
        stamps.append(time.perf_counter())
        return Bpc(v)

    t0 = time.perf_counter()
    oracle.solve(method, A, B, p.b, rtol=0.0, maxit=NU + 1 + 2 * steady, nu_max=NU)
    total = time.perf_counter() - t0
    if "all" in lim:
        lim["all"].restore_original_limits()
    st = np.array(stamps)
    one = float(np.mean(np.diff(st[first:first + steady + 1])))
    allc = float(np.mean(np.diff(st[first + steady:first + 2 * steady + 1])))
    best, best_cores = (allc, cores) if allc < one else (one, 1)
    N = p.N
    scale = N / float(256 ** 3)
    nbytes = iteration_bytes(method, NU, INNER, N)
    return {"value": round(scale / best, 5), "unit": "outer_iters/s", "cores": best_cores, "kind": "oracle",
            "sample": f"{method.upper()} steady iterations {NU + 1}..{NU + steady} (1 thread), "
                      f"{NU + steady + 1}..{NU + 2 * steady} ({cores} threads), same recipe at {n}^3, "
                      f"numpy FP64, {total:.0f} s; value = faster {n}^3 rate x {scale:g} (256^3 unit)",
            f"it_per_s_{n}cube": {"1_thread": round(1.0 / one, 4), f"{cores}_threads": round(1.0 / allc, 4)},
            "algorithmic_GBps": {"1_thread": round(nbytes / one / 1e9, 3),
                                 f"{cores}_threads": round(nbytes / allc / 1e9, 3)},
            "host": {"nproc": cores, "os_cpu_count": os.cpu_count(),
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}}


def _short_kernel_name(name: str) -> str:
    base = name.split("(")[0].replace("void ", "").strip()
    head, sep, tmpl = base.partition("<")
    return head.split("::")[-1] + (("<" + tmpl.replace("pfk::", "")) if sep else "")


def trace_summary(trace_csv: str, kernel: str, skip: int, last: int = 0, count: int = 0) -> str:
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
    if last > 0:
        steady, what = durs[-last:], f"the last {last}"
    elif count > 0:
        steady, what = durs[skip:skip + count], f"dispatches {skip + 1}..{skip + count}"
    else:
        steady, what = durs[skip:], f"dispatch {skip + 1} on"
    if steady:
        steady_sorted = sorted(steady)
        lines.append(f"\n{kernel}: {len(durs)} dispatches; steady state ({what}): "
                     f"{len(steady)} dispatches, mean {sum(steady) / len(steady) / 1e6:.4f} ms, "
                     f"median {steady_sorted[len(steady) // 2] / 1e6:.4f} ms, "
                     f"min {steady_sorted[0] / 1e6:.4f} ms, max {steady_sorted[-1] / 1e6:.4f} ms")
    return "\n".join(lines)


def pmc_summary(csv_path: str, kernel: str = "", last: int = 0) -> str:
    """Mean value per dispatch of each hardware counter, per kernel, from a
    rocprofv3 --pmc counter-collection CSV; for `kernel`, only its last `last`
    dispatches when last > 0 (the steady-state ones of the profiled run)."""
    import csv
    rows = []
    with open(csv_path, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), _short_kernel_name(r["Kernel_Name"]), r["Counter_Name"],
                         float(r["Counter_Value"])))
    rows.sort()
    if kernel and last > 0:
        ids = sorted({d for d, k, _, _ in rows if k == kernel})[-last:]
        keep = set(ids)
        rows = [r for r in rows if r[1] != kernel or r[0] in keep]
    acc = {}
    for d, k, c, v in rows:
        a = acc.setdefault((k, c), [0, 0.0, set()])
        a[1] += v
        a[2].add(d)
    lines = [f"{'kernel':48s} {'counter':12s} {'dispatches':>10s} {'mean per dispatch':>18s}"]
    for (k, c), (_, tot, ids) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{k[:48]:48s} {c:12s} {len(ids):10d} {tot / max(len(ids), 1):18.1f}")
    return "\n".join(lines)


def trace_overlap(trace_csv: str, group_a: str, group_b: str) -> str:
    """How long two groups of kernels (comma-separated name prefixes, short
    names) ran at the same time in a rocprofv3 kernel trace: the busy time of
    each group (union of its kernels' intervals), of both together, and of
    their intersection -- e.g. the kernels of two serving batches that run
    on their own streams."""
    import csv
    pa = tuple(x for x in group_a.split(",") if x)
    pb = tuple(x for x in group_b.split(",") if x)
    ia, ib = [], []
    with open(trace_csv, newline="") as f:
        for r in csv.DictReader(f):
            name = _short_kernel_name(r["Kernel_Name"])
            iv = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
            if name.startswith(pa):
                ia.append(iv)
            elif name.startswith(pb):
                ib.append(iv)

    def union(iv):
        out = []
        for s0, e0 in sorted(iv):
            if out and s0 <= out[-1][1]:
                out[-1][1] = max(out[-1][1], e0)
            else:
                out.append([s0, e0])
        return out

    ua, ub = union(ia), union(ib)
    both = 0
    i = j = 0
    while i < len(ua) and j < len(ub):
        lo, hi = max(ua[i][0], ub[j][0]), min(ua[i][1], ub[j][1])
        if lo < hi:
            both += hi - lo
        if ua[i][1] < ub[j][1]:
            i += 1
        else:
            j += 1
    busy = lambda u: sum(e0 - s0 for s0, e0 in u) / 1e9
    span = (max(e for _, e in ia + ib) - min(s for s, _ in ia + ib)) / 1e9 if ia and ib else 0.0
    return (f"group A ({group_a}): {len(ia)} kernels, busy {busy(ua):.3f} s\n"
            f"group B ({group_b}): {len(ib)} kernels, busy {busy(ub):.3f} s\n"
            f"either busy {busy(union(ia + ib)):.3f} s over a span of {span:.3f} s; "
            f"both at once {both / 1e9:.3f} s")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc-summary":
        sp = argparse.ArgumentParser()
        sp.add_argument("--pmc-summary", required=True, help="rocprofv3 *_counter_collection.csv")
        sp.add_argument("--kernel", default="")
        sp.add_argument("--last", type=int, default=0)
        a = sp.parse_args()
        print(pmc_summary(a.pmc_summary, a.kernel, a.last))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--trace-overlap":
        sp = argparse.ArgumentParser()
        sp.add_argument("--trace-overlap", required=True, help="rocprofv3 *_kernel_trace.csv")
        sp.add_argument("--a", required=True, help="comma-separated kernel name prefixes")
        sp.add_argument("--b", required=True, help="comma-separated kernel name prefixes")
        a = sp.parse_args()
        print(trace_overlap(a.trace_overlap, a.a, a.b))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--trace-summary":
        sp = argparse.ArgumentParser()
        sp.add_argument("--trace-summary", required=True, help="rocprofv3 *_kernel_trace.csv")
        sp.add_argument("--kernel", default="k_pipefcg_update")
        sp.add_argument("--skip", type=int, default=NU + 1)
        sp.add_argument("--last", type=int, default=0, help="use the last N dispatches instead of --skip")
        sp.add_argument("--count", type=int, default=0, help="with --skip: only this many dispatches")
        a = sp.parse_args()
        print(trace_summary(a.trace_summary, a.kernel, a.skip, a.last, a.count))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--method", default="pipefcg", choices=["pipefcg", "fcg"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--detail-out", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for the full record (empty: stderr only)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the FP64 PIPEFCG/FCG pair (for profiler runs)")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 2 GiB device-to-device copy three times (the reference kernel "
                         "for calibrating hardware byte counters)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch geometry")
    ap.add_argument("--tiling", default="",
                    help="TILE_X,STENCIL_TARGET,VECTOR_BLOCKS: this launch geometry for every method of the "
                         "headline pair instead of tuning one (a profiled run then uses the timed run's geometry)")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched workload (after the headline pair)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-batched-solve", action="store_true",
                    help="with --batched-only: steady-state timing only, no solve to tolerance")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="headline pair plus the serving workload (with --serving-requests / --serving-loads)")
    ap.add_argument("--serving-requests", type=int, default=240)
    ap.add_argument("--serving-loads", default="0.9",
                    help="Poisson offered loads as fractions of the measured capacity")
    ap.add_argument("--serving-per-batch", type=int, default=64, help="members per serving batch")
    ap.add_argument("--batched-zc", type=int, default=0,
                    help="z-chunk length (planes) of the batched systems' stencil tiling; 0: the autotuned one")
    # 32: 240-request burst 10.0 s with the operator default (z-marches of one or
    # two planes on these small grids), 9.9 / 9.2 / 8.8 / 12.9 / 12.1 s with 8 /
    # 16 / 32 / 64 / 128 planes
    ap.add_argument("--serving-zc", type=int, default=32,
                    help="z-chunk length (planes) of the serving requests' stencil tiling; 0: the operator default")
    ap.add_argument("--serving-direct", action="store_true",
                    help="serving batches launch kernels directly instead of replaying graphs")
    ap.add_argument("--no-stagnation", action="store_true")
    ap.add_argument("--conv-diff-tts", action="store_true",
                    help="headline plus configuration 3 solved to rtol 1e-8 (256^3, contrasts 1e4 and 1e2)")
    ap.add_argument("--conv-diff-only", action="store_true",
                    help="headline plus the 256^3 convection-diffusion comparison")
    ap.add_argument("--stagnation-only", action="store_true",
                    help="headline plus the noisy-preconditioner stagnation study")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("multi-GPU runs are not part of this build (one GPU per box); use --gpus 1")
        sys.exit(2)

    import torch
    import gen
    import paper_1511_07226_amd as pfk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        src = torch.full((1 << 28,), 1.0, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    log("generating the 256^3 sinker workload")
    prob = gen.config_problem("cfgM", seed=0)
    N = prob.N
    A = pfk.Operator(prob.dim, prob.n, prob.eta)
    B = pfk.Precond(A, "jacobi_pcg", INNER)
    b = torch.as_tensor(prob.b).cuda()
    tuning = {}

    def tune(method):
        # each method is timed with the launch geometry tuned for it
        if args.tiling:
            tx, target, vb = (int(v) for v in args.tiling.split(","))
            tuning[method] = {"tile_x": tx, "stencil_target": target, "vector_blocks": vb, "given": True}
        elif not args.no_autotune:
            tuning[method] = A.autotune(B, method, mmax=NU, reps=3)
            log(f"{method} tiling: {tuning[method]}")

    def rate(method, Bx, **opts):
        t = tuning.get(method)
        if t is not None:
            A.set_tiling(t["tile_x"], t["stencil_target"], t["vector_blocks"])
        S, dt = time_steps(pfk, torch, A, Bx, method, b, args.steps, args.warmup, **opts)
        nbytes = iteration_bytes(method, NU, INNER, N, "block" if Bx.kind == "block_jacobi_pcg" else "global",
                                 Bx.precision == pfk.FP32_BF16COEF)
        return S, {"it_per_s": round(args.steps / dt, 3), "ms_per_step": round(dt / args.steps * 1e3, 4),
                   "algorithmic_GBps": round(nbytes * args.steps / dt / 1e9, 1),
                   "roofline_frac": round(nbytes * args.steps / dt / 1e9 / HBM_PEAK_GBS, 3)}

    results, sessions = {}, {}
    for method in ("pipefcg", "fcg"):
        tune(method)
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
    if args.batched_only:
        args.headline_only = True
        extra["batched_64"] = batched_bench(pfk, torch, args.steps, args.warmup, solve=not args.no_batched_solve,
                                            batch_zc=args.batched_zc)
    if args.stagnation_only:
        args.headline_only = True
        extra["stagnation_study"] = stagnation_study(pfk, torch)
    if args.conv_diff_only:
        args.headline_only = True
        extra["conv_diff_256"] = conv_diff_bench(pfk, torch, args.steps, args.warmup)
    if args.conv_diff_tts:
        args.headline_only = True
        extra["conv_diff_tts"] = conv_diff_tts(pfk, torch)
    loads = tuple(float(v) for v in args.serving_loads.split(",") if v)
    if args.serving_only:
        args.headline_only = True
        extra["serving"] = serving_bench(pfk, torch, nreq=args.serving_requests, loads=loads,
                                         direct=args.serving_direct, per_batch=args.serving_per_batch,
                                         zc=args.serving_zc)
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

        extra["conv_diff_256"] = conv_diff_bench(pfk, torch, args.steps, args.warmup)

    if not args.headline_only and not args.no_stagnation:
        log("stagnation study (section 2.2.1 at scale)")
        extra["stagnation_study"] = stagnation_study(pfk, torch)
    if not args.headline_only:
        log("size sweep: PIPEFCG vs FCG per iteration")
        extra["size_sweep_it_per_s"] = size_sweep(pfk, torch)
    if not args.headline_only and not args.no_batched:
        log("batched workload (64 uneven systems)")
        extra["batched_64"] = batched_bench(pfk, torch, args.steps, args.warmup, batch_zc=args.batched_zc)
        torch.cuda.empty_cache()
    if not args.headline_only and not args.no_serving:
        log("serving workload")
        extra["serving"] = serving_bench(pfk, torch, nreq=args.serving_requests, loads=loads,
                                         direct=args.serving_direct, per_batch=args.serving_per_batch,
                                         zc=args.serving_zc)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle at 128^3, steady state, 1 thread then all host threads)")
        cpu = cpu_baseline(main_m)
        # the GPU at the oracle's sample size, same recipe and launch defaults
        pc = gen.config_problem("cfgM", seed=0, n=128)
        Ac = pfk.Operator(pc.dim, pc.n, pc.eta)
        Sx, dt = time_steps(pfk, torch, Ac, pfk.Precond(Ac, "jacobi_pcg", INNER), main_m,
                            torch.as_tensor(pc.b).cuda(), args.steps, args.warmup)
        Sx.close()
        cpu["gpu_it_per_s_128cube"] = round(args.steps / dt, 1)
        del pc, Ac

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
                   "unknowns": N, "method": main_m, "nu_max": NU, "inner_its": INNER,
                   "launch_geometry": tuning.get(main_m, "default")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": update_traffic_bytes() if main_m == "pipefcg" else None,
                     "kernel": upd_name, "avg_ms": round(avg_ms, 4),
                     "algorithmic_bytes_per_launch": int(upd_bytes)},
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
    # everything goes to the detail record (a file and one stderr line); stdout
    # ends with the compact headline line
    detail = json.dumps(out)
    path = args.detail_out
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            f.write(detail + "\n")
        log(f"detail record written to {path}")
    print("[bench] detail " + detail, file=sys.stderr, flush=True)
    head = {k: out[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    head["config"] = {k: out["config"][k] for k in ("workload", "unknowns", "method", "nu_max", "inner_its")}
    head["roofline"] = out["roofline"]
    head["cpu_baseline"] = compact_cpu(cpu)
    head["compare"] = compact_compare(out["compare"], other)
    print(json.dumps(head, separators=(",", ":")), flush=True)


def compact_cpu(cpu):
    if cpu is None:
        return None
    keep = ("value", "unit", "cores", "kind", "sample", "gpu_it_per_s_128cube")
    c = {k: cpu[k] for k in keep if k in cpu}
    c["it_per_s_128cube"] = next((v for k, v in cpu.items() if k.startswith("it_per_s_")), None)
    c["nproc"] = cpu.get("host", {}).get("nproc")
    return c


def compact_compare(cmp, other):
    """The headline comparisons in a few hundred bytes: rates, ratios,
    convergence counts and latencies (the full record is the detail line)."""
    def rate(d):
        return d.get("it_per_s") if isinstance(d, dict) else None

    c = {f"{other}_it_per_s": rate(cmp[other]), "pipelined_over_unpipelined": cmp["pipelined_over_unpipelined"],
         "GBps_whole_iteration": cmp["algorithmic_GBps_whole_iteration"]}
    # (the host-synchronised FCG baseline stays in the detail line)
    for k in ("pipefcg_mixed", "fcg_mixed", "pipefcg_block", "fcg_block",
              "pipefcg_block_mixed", "fcg_block_mixed"):
        if k in cmp:
            c[k] = rate(cmp[k])
    cd = cmp.get("conv_diff_256")
    if cd:
        c["conv_diff_256_it_per_s"] = {m: rate(cd[m]) for m in ("pipefgmres", "fgmres", "pipegcr", "pipegcr_w", "gcr")
                                       if m in cd}
    tts = cmp.get("time_to_solution_rtol1e-8")
    if tts:
        c["tts_128_s"] = {k: v["seconds"] for k, v in tts.items() if isinstance(v, dict)}
    bt = cmp.get("batched_64")
    if bt:
        t = bt.get("time_to_solution", {})
        c["batched_64"] = {"pipefcg_batch_it_per_s": bt.get("pipefcg_batch_iters_per_s"),
                           "fcg_batch_it_per_s": bt.get("fcg_batch_iters_per_s"),
                           "pipefcg_persistent_it_per_s": bt.get("pipefcg_persistent_batch_iters_per_s"),
                           "speedup_vs_one_at_a_time": bt.get("batching_speedup"),
                           "solve_s": t.get("seconds"), "converged": t.get("converged"),
                           "max_true_rel": (float(f"{t['max_true_rel_resid']:.4g}")
                                            if t.get("max_true_rel_resid") is not None else None)}
    sv = cmp.get("serving")
    if sv:
        def ms(v):
            return round(v) if isinstance(v, (int, float)) else v

        row = {"capacity": {k: (ms(sv["burst"][k]) if k.endswith("_ms") else sv["burst"][k])
                            for k in ("converged_solves_per_s", "p50_ms", "p99_ms", "converged", "requests")}}
        for f, r in sv.get("poisson", {}).items():
            row[f] = [r["converged_solves_per_s"], ms(r["p50_ms"]), ms(r["p99_ms"])]
        c["serving"] = row
    sw = cmp.get("size_sweep_it_per_s")
    if sw:
        c["size_sweep_pipe_over_unpipe"] = {k: v["pipelined_over_unpipelined"] for k, v in sw.items()}
    return c


if __name__ == "__main__":
    main()
