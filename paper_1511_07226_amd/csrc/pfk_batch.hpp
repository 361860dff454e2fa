// Batched kernels: one launch advances one phase of an outer iteration for
// every system of a batch.
//
// Each system keeps its own operator, preconditioner, workspace and device
// SolveState (exactly those of a single solve); a device table of BSys
// records holds the pointers and launch geometry of each.  A phase's launch
// is the concatenation of every system's own launch of that phase: system s
// owns workgroups [off[s], off[s+1]) (ranges start at multiples of 8, so the
// XCD-aware tile order of the stencil engine carries over), finds its record
// by binary search and runs the same device body as the single-system kernel
// with its index inside the range.  Systems of different sizes therefore
// share launches without any per-system kernel boundary, and a system that
// has stopped (converged, failed, or waiting for a host decision) returns at
// once in every phase.
#pragma once
#include "pfk_gmres.hpp"

namespace pfk {

// Per-system arguments of the batched phases.
struct BSys {
  long long N;
  Grid g;                 // outer operator
  GridM gm;               // inner operator of the mixed-precision block preconditioner
  StencilGeom sg;         // the system's stencil launch geometry
  int Pv, Ps;             // its vector / stencil workgroup counts
  int bj_wx, bj_wy, bj_n; // its block-preconditioner launch (workgroups along x, y; total)
  int pc_k;               // inner iterations
  PcOutDesc pd;           // where B(v) comes from (input vectors, the inner solve's buffers)
  void* pc_pbase;         // global inner solves' work vectors (arithmetic type of the inner sweeps):
  long long pc_ldp;       //   PCG directions p_1 .. p_k (pc_ldp elements apart), A p, residual;
  void *pc_q, *pc_rho;    //   GMRES: pc_q holds w~
  double *part_pc0, *part_pc1;   // their partial sums
  Window P, S, Q, Z;      // direction windows (method-dependent roles, as in a single solve)
  double *x, *r, *u, *w, *m, *n, *z, *x0;
  double *part_main, *part_a, *part_b;
  SolveState* st;
  double* hist;
};

// Phases: workgroup-range tables, one per launch shape.
enum BPhase { kBpVec = 0, kBpSten = 1, kBpBlk = 2, kBpOne = 3, kBpCount = 4 };

// System owning workgroup b: the largest s with off[s] <= b.
__device__ __forceinline__ int batch_find(const int* off, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---- PIPEFCG ------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) kb_pipefcg_update(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  pipefcg_update_body(bk, d.N, d.P, d.S, d.Q, d.Z, d.x, d.r, d.u, d.w, d.m, d.n, d.part_main, d.st, 0);
}

__global__ void __launch_bounds__(kBlock) kb_pipefcg_scalars(const BSys* sys) {
  const BSys& d = sys[blockIdx.x];
  pipefcg_scalars_body(Blk{0, 1}, d.part_main, d.Pv, d.st, d.hist);
}

// m = u + B(w - r), n = A m (PIPEFCG); wbar = A B(zbar) (PIPEFGMRES, O unused).
// Every member has the same inner kind and storage, so the host picks the
// instantiation (K, F32) as for a single solve, and each carries only its
// own registers (K < 0: NONE, JACOBI, FP64 GMRES, decided at run time).
template <int K, int F32>
__global__ void __launch_bounds__(kBlock) kb_apply_pc_out(const BSys* sys, const int* off, int nsys, int pipefcg) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Ps};
  if (bk.id >= bk.n) return;   // padding of the range
  if (!wg_running(d.st)) return;
  if (pipefcg)
    apply_pc_out_t<K, F32, false>(bk, d.g, d.sg, d.pd, d.u, 1.0, d.m, d.n, 0, nullptr, d.part_b, d.st);
  else
    apply_pc_out_t<K, F32, false>(bk, d.g, d.sg, d.pd, nullptr, 0.0, nullptr, d.z, 0, nullptr, d.part_b, d.st);
}

// ---- the global inner solves of every system ----------------------------------
// The same phases a single solve launches (pfk_pc.hpp), each over all members:
// k-step Jacobi-PCG as A_1, then (B_j, A_{j+1}) for j < k; k-step right-Jacobi
// GMRES as GF_j for j < k, then GE.  Every member of a batch has
// the same inner kind, precision and step count k.  T: the inner arithmetic
// (FP32 sweeps run on the BF16 viscosity copy).
template <class T, class F>
__device__ __forceinline__ void with_inner_grid(const BSys& d, F&& f) {
  if constexpr (sizeof(T) == 4) f(d.gm);
  else f(d.g);
}

template <class T>
__global__ void __launch_bounds__(kBlock) kb_pcg_a1(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Ps};
  if (bk.id >= bk.n) return;   // padding of the range
  const PcOutDesc& pd = d.pd;
  with_inner_grid<T>(d, [&](const auto& g) {
    pcg_a1_body<T>(bk, g, d.sg, (const T*)pd.dinv_in, pd.X1, pd.c1, pd.X2, pd.c2, (T*)d.pc_pbase, (T*)d.pc_q,
                   d.part_pc0, d.st);
  });
}

// B_j: rho -= alpha q, the last one also y (reads A_j's partials, PC0; writes PC1)
template <class T>
__global__ void __launch_bounds__(kBlock) kb_pcg_b(const BSys* sys, const int* off, int nsys, int j) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  const PcOutDesc& pd = d.pd;
  pcg_b_body<T>(bk, j, d.pc_k, d.N, (const T*)pd.dinv_in, pd.X1, pd.c1, pd.X2, pd.c2, (const T*)d.pc_pbase,
                d.pc_ldp, (const T*)d.pc_q, (T*)d.pc_rho, (T*)const_cast<void*>(pd.y), d.part_pc0, d.Ps,
                d.part_pc1, d.st);
}

// A_{j+1}: p_{j+1} = D^-1 rho + beta p_j, q = A p_{j+1} (reads PC1, writes PC0)
template <class T>
__global__ void __launch_bounds__(kBlock) kb_pcg_a(const BSys* sys, const int* off, int nsys, int j) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Ps};
  if (bk.id >= bk.n) return;   // padding of the range
  const PcOutDesc& pd = d.pd;
  const T* pj = (const T*)d.pc_pbase + (long long)(j - 1) * d.pc_ldp;
  T* pn = (T*)d.pc_pbase + (long long)j * d.pc_ldp;
  with_inner_grid<T>(d, [&](const auto& g) {
    pcg_a_body<T>(bk, j + 1, g, d.sg, (const T*)pd.dinv_in, (const T*)d.pc_rho, pj, pn, (T*)d.pc_q,
                  d.part_pc1, d.Pv, d.part_pc0, d.st);
  });
}

// The inner GMRES of every member (GF_j and GE as in a single solve; w~
// and the partials alternate between two buffers).  Velocities are loaded
// where used in every member (the load-ahead form of a single solve rounds
// alike).
template <class T>
__device__ __forceinline__ T* batch_gm_w(const BSys& d, int j) {
  const PcOutDesc& pd = d.pd;
  return (j & 1) ? (T*)const_cast<void*>(pd.vbase) + (long long)pd.k * pd.ldv : (T*)d.pc_q;
}
__device__ __forceinline__ double* batch_gm_part(const BSys& d, int j) {
  return (j & 1) ? d.part_pc1 : d.part_pc0;
}
// GF_j: reads GF_{j-1}'s partials, writes its own
template <class T, int J, bool WW>
__global__ void __launch_bounds__(kBlock) kb_gmpc_fused(const BSys* sys, const int* off, int nsys, int j) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Ps};
  if (bk.id >= bk.n) return;   // padding of the range
  const PcOutDesc& pd = d.pd;
  const T* wp = j > 0 ? batch_gm_w<T>(d, j - 1) : nullptr;
  with_inner_grid<T>(d, [&](const auto& g) {
    gmpc_fused_body<T, std::decay_t<decltype(g)>, 0, J, WW>(
        bk, j, pd.k, g, d.sg, (const T*)pd.dinv_in, pd.X1, pd.c1, pd.X2, pd.c2, (T*)const_cast<void*>(pd.vbase),
        pd.ldv, wp, batch_gm_w<T>(d, j), batch_gm_part(d, j + 1), d.Ps, batch_gm_part(d, j), d.st);
  });
}

// GE: one workgroup per member (reads GF_{k-1}'s partials)
__global__ void __launch_bounds__(kBlock) kb_gmpc_finish(const BSys* sys, int nsys) {
  const BSys& d = sys[blockIdx.x];
  gmpc_finish_body(d.pd.k, batch_gm_part(d, d.pd.k - 1), d.Ps, d.st);
}

// ---- the block-Jacobi inner solve of every system -----------------------------
template <class T, int D3>
__global__ void __launch_bounds__(kBlock) kb_block_pcg(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.bj_n};
  if (bk.id >= bk.n) return;   // padding of the range
  const PcOutDesc& pd = d.pd;
  if constexpr (sizeof(T) == 4)
    block_pcg_body<float, GridM, D3>(bk, d.gm, d.bj_wx, d.bj_wy, d.pc_k, pd.X1, pd.c1, pd.X2, pd.c2,
                                     (float*)const_cast<void*>(pd.y), d.st);
  else
    block_pcg_body<double, Grid, D3>(bk, d.g, d.bj_wx, d.bj_wy, d.pc_k, pd.X1, pd.c1, pd.X2, pd.c2,
                                     (double*)const_cast<void*>(pd.y), d.st);
}

// ---- FCG ----------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) kb_fcg_xr(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  fcg_xr_body(bk, d.N, d.P, d.S, d.x, d.r, d.st);
}

// u = B(r) with the first reduction (<u,r>, <u,u>, <r,r>, <u, s_d>)
__global__ void __launch_bounds__(kBlock) kb_fcg_multidot(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  multidot_body(bk, d.N, 0, 1, d.pd, nullptr, d.u, d.r, d.S, d.part_main, d.st);
}

__global__ void __launch_bounds__(kBlock) kb_cg_scalars1(const BSys* sys) {
  const BSys& d = sys[blockIdx.x];
  cg_scalars1_body(Blk{0, 1}, 0, d.part_main, d.Pv, d.st, d.hist);
}

__global__ void __launch_bounds__(kBlock) kb_fcg_maxpy(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  fcg_maxpy_body(bk, d.N, d.P, d.u, d.st);
}

__global__ void __launch_bounds__(kBlock) kb_fcg_apply(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Ps};
  if (bk.id >= bk.n) return;   // padding of the range
  fcg_apply_body(bk, d.g, d.sg, d.P, d.S, d.part_a, d.st);
}

__global__ void __launch_bounds__(kBlock) kb_cg_scalars2(const BSys* sys) {
  const BSys& d = sys[blockIdx.x];
  cg_scalars2_body(Blk{0, 1}, 0, 0, d.part_a, d.Ps, d.st);
}

// ---- PIPEFGMRES ---------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) kb_pgm_update(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  // P: basis p, S: u~, Q: zbar; qbar = B(zbar) of the previous column from d.pd
  pgm_update_body(bk, d.N, d.P, d.S, d.Q, d.pd, d.z, d.m, d.part_main, d.st);
}

__global__ void __launch_bounds__(kBlock) kb_pgm_scalars(const BSys* sys) {
  const BSys& d = sys[blockIdx.x];
  pgm_scalars_body(Blk{0, 1}, d.part_main, d.Pv, d.st, d.hist);
}

__global__ void __launch_bounds__(kBlock) kb_gm_update_x(const BSys* sys, const int* off, int nsys) {
  const int s = batch_find(off, nsys, (int)blockIdx.x);
  const BSys& d = sys[s];
  const Blk bk{(int)blockIdx.x - off[s], d.Pv};
  if (bk.id >= bk.n) return;   // padding of the range
  gm_update_x_body(bk, d.N, d.S, d.x0, d.x, d.st);
}

// ---- status of every system in one copy ----------------------------------------
__global__ void __launch_bounds__(kBlock) kb_gather_status(const BSys* sys, int nsys, int* out) {
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < nsys; s += gridDim.x * kBlock) {
    out[2 * s] = read_status(sys[s].st);
    out[2 * s + 1] = sys[s].st->it;
  }
}

}  // namespace pfk

namespace pfk {

// ---- persistent form ----------------------------------------------------------
// One cooperative launch runs `iters` outer iterations of every member: the
// phases are separated by a grid barrier instead of kernel boundaries, and
// inside a phase the workgroups take the phase's work items (the concatenated
// per-member ranges of the phased form) round robin.  The reduction finish of
// the PIPE methods shares a phase with the preconditioner, so it costs no
// barrier of its own; FCG's two finishes each sit between two barriers.
//
// Barrier: two-level arrival (one counter per XCD slot, workgroup b arriving
// on slot b mod 8, whose last arrival arrives at the top counter) and a
// generation word in device memory.  Stores of the phase are ordered before
// the arrival by the workgroup barrier (which waits for each wave's stores)
// and an agent-scope release fence; the waiting side polls the generation
// with relaxed loads (no cache invalidation per poll, so waiting workgroups do
// not disturb the ones still working) and acquires once it changes.  The wait
// is bounded: a workgroup that polls more than `limit` times sets `abort`,
// and every workgroup that sees it leaves the kernel, so every wave exits.
struct GridBarrier {
  unsigned slot[8][16];   // arrival counters, one 64-byte line each
  unsigned top;
  unsigned gen;
  int abort;
  int pad;
  long long limit;        // polls before a wait gives up
};
constexpr long long kBarrierSpins = 1LL << 24;   // ~1 s with the 64-cycle sleep

__device__ __forceinline__ bool grid_barrier(GridBarrier* b, unsigned nblocks) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned lane = blockIdx.x & 7u;
    // workgroups in this slot: those b < nblocks with b mod 8 == lane (nblocks is a multiple of 8)
    const unsigned per_slot = nblocks / 8u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the phase's stores, before arriving
    bool last = false;
    const unsigned a = __hip_atomic_fetch_add(&b->slot[lane][0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (a == per_slot) {
      __hip_atomic_store(&b->slot[lane][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned t = __hip_atomic_fetch_add(&b->top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
      last = (t == 8u);
    }
    if (last) {
      __hip_atomic_store(&b->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > b->limit) {
          __hip_atomic_store(&b->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the other workgroups' stores of the phase
    if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// PC: 0 = no inner-solve kernel (NONE, JACOBI), 1 = block PCG in FP64, 2 = in FP32.
template <int PC, int D3>
__device__ __forceinline__ void kp_block_items(const BSys* sys, const int* off, int nsys, int tot, int first,
                                               int stride) {
  if constexpr (PC != 0) {
    for (int it = first; it < tot; it += stride) {
      const int s = batch_find(off, nsys, it);
      const BSys& d = sys[s];
      const Blk bk{it - off[s], d.bj_n};
      if (bk.id >= bk.n) continue;
      const PcOutDesc& pd = d.pd;
      if constexpr (PC == 2)
        block_pcg_body<float, GridM, D3>(bk, d.gm, d.bj_wx, d.bj_wy, d.pc_k, pd.X1, pd.c1, pd.X2, pd.c2,
                                         (float*)const_cast<void*>(pd.y), d.st);
      else
        block_pcg_body<double, Grid, D3>(bk, d.g, d.bj_wx, d.bj_wy, d.pc_k, pd.X1, pd.c1, pd.X2, pd.c2,
                                         (double*)const_cast<void*>(pd.y), d.st);
    }
  }
}

// Apply F(d, bk) to every work item of a phase this workgroup owns.
template <class F>
__device__ __forceinline__ void kp_items(const BSys* sys, const int* off, int nsys, int tot, int which, F&& f) {
  for (int it = (int)blockIdx.x; it < tot; it += (int)gridDim.x) {
    const int s = batch_find(off, nsys, it);
    const BSys& d = sys[s];
    const int count = which == kBpVec ? d.Pv : d.Ps;
    const Blk bk{it - off[s], count};
    if (bk.id >= bk.n) continue;
    f(d, bk);
  }
}

template <int M, int PC, int D3>
__global__ void __launch_bounds__(kBlock)
kp_batch(const BSys* sys, const int* offs, int nsys, int tot_vec, int tot_sten, int tot_blk, int iters,
         GridBarrier* bar) {
  const int* ov = offs + kBpVec * (nsys + 1);
  const int* os = offs + kBpSten * (nsys + 1);
  const int* ob = offs + kBpBlk * (nsys + 1);
  const unsigned G = gridDim.x;
  for (int k = 0; k < iters; ++k) {
    if constexpr (M == PFK_PIPEFCG) {
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        pipefcg_update_body(bk, d.N, d.P, d.S, d.Q, d.Z, d.x, d.r, d.u, d.w, d.m, d.n, d.part_main, d.st, 0);
      });
      if (!grid_barrier(bar, G)) return;
      // the reduction finish of every member beside the inner solves
      for (int s = (int)blockIdx.x; s < nsys; s += (int)G)
        pipefcg_scalars_body(Blk{0, 1}, sys[s].part_main, sys[s].Pv, sys[s].st, sys[s].hist);
      kp_block_items<PC, D3>(sys, ob, nsys, tot_blk, (int)((blockIdx.x + G - (unsigned)(nsys % (int)G)) % G), (int)G);
      if (!grid_barrier(bar, G)) return;
      kp_items(sys, os, nsys, tot_sten, kBpSten, [&](const BSys& d, Blk bk) {
        apply_pc_out_body(bk, d.g, d.sg, d.pd, d.u, 1.0, d.m, d.n, 0, nullptr, d.part_b, d.st);
      });
      if (!grid_barrier(bar, G)) return;
    } else if constexpr (M == PFK_FCG) {
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        fcg_xr_body(bk, d.N, d.P, d.S, d.x, d.r, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      if constexpr (PC != 0) {
        kp_block_items<PC, D3>(sys, ob, nsys, tot_blk, (int)blockIdx.x, (int)G);
        if (!grid_barrier(bar, G)) return;
      }
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        multidot_body(bk, d.N, 0, 1, d.pd, nullptr, d.u, d.r, d.S, d.part_main, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      for (int s = (int)blockIdx.x; s < nsys; s += (int)G)
        cg_scalars1_body(Blk{0, 1}, 0, sys[s].part_main, sys[s].Pv, sys[s].st, sys[s].hist);
      if (!grid_barrier(bar, G)) return;
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        fcg_maxpy_body(bk, d.N, d.P, d.u, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      kp_items(sys, os, nsys, tot_sten, kBpSten, [&](const BSys& d, Blk bk) {
        fcg_apply_body(bk, d.g, d.sg, d.P, d.S, d.part_a, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      for (int s = (int)blockIdx.x; s < nsys; s += (int)G)
        cg_scalars2_body(Blk{0, 1}, 0, 0, sys[s].part_a, sys[s].Ps, sys[s].st);
      if (!grid_barrier(bar, G)) return;
    } else {   // PIPEFGMRES
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        pgm_update_body(bk, d.N, d.P, d.S, d.Q, d.pd, d.z, d.m, d.part_main, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      for (int s = (int)blockIdx.x; s < nsys; s += (int)G)
        pgm_scalars_body(Blk{0, 1}, sys[s].part_main, sys[s].Pv, sys[s].st, sys[s].hist);
      kp_block_items<PC, D3>(sys, ob, nsys, tot_blk, (int)((blockIdx.x + G - (unsigned)(nsys % (int)G)) % G), (int)G);
      if (!grid_barrier(bar, G)) return;
      kp_items(sys, os, nsys, tot_sten, kBpSten, [&](const BSys& d, Blk bk) {
        apply_pc_out_body(bk, d.g, d.sg, d.pd, nullptr, 0.0, nullptr, d.z, 0, nullptr, d.part_b, d.st);
      });
      if (!grid_barrier(bar, G)) return;
      kp_items(sys, ov, nsys, tot_vec, kBpVec, [&](const BSys& d, Blk bk) {
        gm_update_x_body(bk, d.N, d.S, d.x0, d.x, d.st);
      });
      if (!grid_barrier(bar, G)) return;
    }
  }
}

}  // namespace pfk
