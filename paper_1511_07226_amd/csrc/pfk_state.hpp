// Device-resident solver state: the scalar block every kernel of a solve reads
// (status, iteration counters, alpha/beta/eta of the direction window, the
// Hessenberg least-squares data of the GMRES family) and the preconditioner's
// per-application scalars.  It lives in the caller's workspace; the host only
// reads it (asynchronously) between graph launches.
#pragma once
#include "pfk_device.hpp"

namespace pfk {

enum Status : int {
  kRunning = 0,
  kConverged = 1,    // recurred residual below tolerance; true residual still to check
  kBreakdown = 2,    // norm breakdown: restart from the current x
  kMaxit = 3,
  kBreakdown0 = 4,   // breakdown of the initial direction: unrecoverable
  kCycleEnd = 5,     // GMRES family: restart length reached
  kNonfinite = 6,
  kDone = 7,         // true residual confirmed below tolerance
  kGap = 8,          // true residual above tolerance: restart from x
};

constexpr int kMaxInner = 32;      // largest inner iteration count of a preconditioner

struct PcScalars {                 // one inner solve's scalars, indexed by inner step
  double gamma[kMaxInner + 2];
  int stopped[kMaxInner + 2];
  double alpha[kMaxInner + 2];    // inner PCG step lengths (in the inner arithmetic type)
  // inner GMRES: Hessenberg h(i,j) at h[j*(kMaxInner+1)+i], basis scales
  // (V_j = vs[j] * stored vector j), active columns
  double h[(kMaxInner + 1) * kMaxInner];
  double vs[kMaxInner + 1];
  double beta0;
  int ncol;
  // its least-squares result: B(v) = D^-1 sum_q cf[q] (stored q), q < nv
  double cf[kMaxInner + 1];
  int nv;
  // noisy preconditioner: applications of B this solve has used so far, and
  // whether the current phase runs
  unsigned long long ndraws;
  int noise_live;
};

constexpr int kMaxInnerGmres = 8;  // inner GMRES steps supported

struct SolveState {
  int status;
  int it;            // iterations completed since the start of the solve
  int j;             // CG/CR: index of the newest direction since the last (re)start
  int nu_max;        // window length (CG/CR) or restart length (GMRES)
  int trunc;         // truncation rule: 0 min(j,nu_max), 1 max(1, j mod (nu_max+1)), 2 min(j, j mod nu_max + 1)
  int maxit;
  int force_it;      // test hook: iteration at which a breakdown is forced (one-shot), -1 off
  int hist_started;
  int nu;            // number of window directions of the current update
  int bzero;         // b == 0: the solve is finished with x = 0
  double tol;        // rtol * ||b||_2
  double alpha;      // step length of the next solution update
  double gamma, delta, rho, eta_new;
  double sigma;      // PIPEFGMRES shift
  double true_res;
  double bnorm;      // ||b||_2
  int norm;          // CG/CR types: 1 tests the natural norm sqrt|gamma| instead of ||r||_2
  int stall;         // CG/CR types: stagnation restart window K (0 off)
  int nat_started;   // natural-norm history entry 0 recorded (first start-up)
  int nt;            // vector kernels use nontemporal accesses (working set far beyond the caches)
  double rtol;
  double ntol;       // rtol * natural norm of the first start-up
  double* nhist;     // natural-norm history (device), or null
  unsigned long long* tstamp;   // device clock per history entry, or null
  double eta_ring[kNuMax];   // eta of direction d at slot d mod nu_max
  double beta[kNuMax];       // beta of the current update, window order (oldest first)
  // GMRES family (restart length m <= kNuMax)
  int col;           // Arnoldi columns finished in this cycle
  int pend;          // 1: the cycle ended and x = x0 + U y is (re)applied by k_gm_update_x
  int ycols;         // columns of y
  int pad1;
  double beta0;      // ||r_0|| of the cycle
  double hbar[kNuMax + 1];
  double hn;         // norm of the new basis vector (h_{i,i-1})
  double inv_hn;     // 1 / hn, scales the next basis vectors
  double R[(kNuMax + 1) * kNuMax];   // rotated Hessenberg, column-major (m+1) x m
  double cs[kNuMax], sn[kNuMax], g[kNuMax + 1], y[kNuMax];
  PcScalars pc;
};

__host__ __device__ inline int trunc_nu(int rule, int j, int numax) {
  if (j < 1) return 0;
  if (rule == 1) {
    const int m = j % (numax + 1);
    return m < 1 ? 1 : m;
  }
  if (rule == 2) {
    const int m = j % numax + 1;
    return m < j ? m : j;
  }
  return j < numax ? j : numax;
}

// The device's constant-rate wall clock at history entry i (opts.timestamps).
__device__ __forceinline__ void log_time(SolveState* st, int i) {
  if (st->tstamp) st->tstamp[i] = wall_clock64();
}

// Stagnation (option stall_window K, CG/CR types): at least K iterations since
// the (re)start and the newest recurred residual above half of the one K
// iterations back; the solve then restarts from x as after a residual gap.
__device__ __forceinline__ bool stalled(const SolveState* st, const double* hist, int it, int j, double res) {
  return st->stall > 0 && j >= st->stall && res > 0.5 * hist[it - st->stall];
}

__device__ __forceinline__ int read_status(const SolveState* st) {
  return __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether the solve runs, as one value for the whole workgroup (thread 0
// reads, a barrier shares it).  Every kernel and device body tests the status
// this way on entry: the preconditioner and operator kernels of a pipelined
// method run on one stream while the scalar kernel on the other may change
// the status, and a per-thread read could send the waves of one workgroup to
// different sides of the body's barriers (inside a persistent launch an early
// return does not even end the wave).
__device__ __forceinline__ bool wg_running(const SolveState* st) {
  __shared__ int s_run;
  __syncthreads();
  if (threadIdx.x == 0) s_run = read_status(st) == kRunning;
  __syncthreads();
  return s_run != 0;
}

// A value that another workgroup of the same launch may be writing, read once
// for the whole workgroup (thread 0 reads, a barrier shares it), so all its
// waves take the same side of the barriers that follow.
__device__ __forceinline__ int wg_load(const int* p) {
  __shared__ int s_val;
  __syncthreads();
  if (threadIdx.x == 0) s_val = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return s_val;
}

}  // namespace pfk
