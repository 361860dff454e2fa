// Outer kernels of the CG family: FCG (Alg. 2) and PIPEFCG (Alg. 8), plus the
// kernels every method shares (solve set-up, r = b - A x, the operator
// applied to a combination of vectors, the true-residual check).
//
// Direction windows are ring buffers: direction d (counted from the last
// (re)start) lives in slot d mod nu_max of each window array, whose vectors
// are `ld` doubles apart.  The scalar recurrences run in single-workgroup
// kernels (k_*_scalars) that leave their results in SolveState; the vector
// kernels read them there.  Every kernel returns at once when the solve is no
// longer running, so iterations enqueued after convergence change nothing.
#pragma once
#include "pfk_pc.hpp"

namespace pfk {

struct Window {
  double* base;
  long long ld;
  __device__ __forceinline__ double* slot(int s) const { return base + (long long)s * ld; }
};

// ---------------------------------------------------------------------------
// Shared kernels
// ---------------------------------------------------------------------------
__global__ void k_setup(SolveState* st, double tol, int maxit, int nu_max, int trunc, int force_it,
                        double sigma, int norm, double* nhist, int nt, unsigned long long* tstamp, int stall) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->nt = nt;
  st->status = kRunning;
  st->it = 0;
  st->j = 0;
  st->nu_max = nu_max;
  st->trunc = trunc;
  st->maxit = maxit;
  st->force_it = force_it;
  st->hist_started = 0;
  st->nu = 0;
  st->tol = tol;
  st->alpha = 0.0;
  st->sigma = sigma;
  st->true_res = 0.0;
  st->col = 0;
  st->bzero = 0;
  st->bnorm = 0.0;
  st->pc.ndraws = 0;
  st->pc.noise_live = 0;
  st->norm = norm;
  st->nat_started = 0;
  st->rtol = 0.0;
  st->ntol = 0.0;
  st->nhist = nhist;
  st->tstamp = tstamp;
  st->stall = stall;
}

// Natural norm sqrt|gamma| (section 5: the residual norm CG/CR types have
// without an extra reduction; gamma = <u, r> or <r, A u>).  The first
// start-up records entry 0 and the tolerance rtol * entry 0; every iteration
// logs its entry, and natural_test says whether it passes.
__device__ __forceinline__ void natural_start(SolveState* st, double gamma) {
  if (st->nat_started) return;
  st->nat_started = 1;
  const double v = sqrt(fabs(gamma));
  if (st->nhist) st->nhist[0] = v;
  st->ntol = st->rtol * v;
}
__device__ __forceinline__ double natural_log(SolveState* st, int it, double gamma) {
  const double v = sqrt(fabs(gamma));
  if (st->nhist) st->nhist[it] = v;
  return v;
}
// The convergence test of the chosen norm (res = recurred ||r||_2).
__device__ __forceinline__ bool converged_test(const SolveState* st, double res, double nat) {
  return st->norm ? nat <= st->ntol : res <= st->tol;
}

// Start (or restart) a cycle from the current x: the pipeline is flushed.
__global__ void k_restart(SolveState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->status = st->bzero ? kDone : kRunning;
  st->j = 0;
  st->nu = 0;
  st->col = 0;
}

// r = b - A x, partial <r, r>; optionally a copy x0 = x (GMRES cycle start).
__global__ void __launch_bounds__(kBlock)
k_residual(Grid g, StencilGeom sg, const double* __restrict__ b, const double* __restrict__ x,
           double* __restrict__ r, double* part, double* __restrict__ x0) {
  double acc[1] = {0.0};
  const auto in = stencil_in([&](long long t) { return x[t]; });
  auto sink = [&](long long idx, double xc, double Au) {
    if (x0 != nullptr) x0[idx] = xc;
    const double rv = b[idx] - Au;
    r[idx] = rv;
    acc[0] += rv * rv;
  };
  stencil_march<double>(g, sg, in, sink);
  block_partials<1>(acc, 1, part, sg.blocks());
}

// y = A x (operator checks; PIPEGCR's w = A u when st is given).  k_apply_cv
// is the same body for operators with face velocities, which the stencil
// then loads ahead of use.
template <bool CV>
__device__ __forceinline__ void apply_body(const Grid& g, const StencilGeom& sg, const double* __restrict__ x,
                                           double* __restrict__ y, const SolveState* st) {
  if (st != nullptr && !wg_running(st)) return;
  const auto in = stencil_in([&](long long t) { return x[t]; });
  auto sink = [&](long long idx, double, double Au) { y[idx] = Au; };
  stencil_march<double, CV>(g, sg, in, sink);
}
__global__ void __launch_bounds__(kBlock)
k_apply(Grid g, StencilGeom sg, const double* __restrict__ x, double* __restrict__ y, const SolveState* st) {
  apply_body<false>(g, sg, x, y, st);
}
__global__ void __launch_bounds__(kBlock)
k_apply_cv(Grid g, StencilGeom sg, const double* __restrict__ x, double* __restrict__ y, const SolveState* st) {
  apply_body<true>(g, sg, x, y, st);
}

// O = c3*X3 + B(v) at every node, N = A O.  With dots = 1: partials <O, R>,
// <O, N>; with dots = 2: <N, R>, <N, N>.
// Used for u_0/w_0 and m_0/n_0 of PIPEFCG's start-up and for m_i, n_i in its
// loop (m_i = u_i + B(w_i - r_i), n_i = A m_i).  K: the inner solve's
// output kind fixed at compile time (K < 0: decided at run time); GM: the
// run-time path loads an FP32 inner GMRES output ahead (gm_raw_in).
template <int K, int F32, bool GM = false>
__device__ __forceinline__ void apply_pc_out_t(Blk bk, const Grid& g, const StencilGeom& sg, const PcOutDesc& pd,
                                               const double* X3, double c3, double* __restrict__ O,
                                               double* __restrict__ Nout, int dots, const double* __restrict__ R,
                                               double* part, SolveState* st) {
  const PcOut pc = make_pc_out(pd, &st->pc);
  const bool nt = st->nt != 0;
  double acc[2] = {0.0, 0.0};
  auto sink = [&](long long idx, double mc, double nv) {
    if (nt) {
      if (O != nullptr) stnt(O + idx, mc);
      stnt(Nout + idx, nv);
    } else {
      if (O != nullptr) O[idx] = mc;
      Nout[idx] = nv;
    }
    if (dots == 1) {            // <O, R>, <O, N>
      acc[0] += mc * R[idx];
      acc[1] += mc * nv;
    } else if (dots == 2) {     // <N, R>, <N, N>
      acc[0] += nv * R[idx];
      acc[1] += nv * nv;
    }
  };
  if constexpr (K == kPcBlockPcg || K == kPcJacobiPcg) {
    // the inner solve's stored output (and X3) are loaded ahead; the value is
    // PcOut::at's arithmetic, plus c3*X3
    using W = typename std::conditional<F32 != 0, float, double>::type;
    struct RawPc { W y, p; double x3; };
    const W* yw = static_cast<const W*>(pc.y);
    const W* pw = static_cast<const W*>(pc.pk);
    const bool ly = K == kPcBlockPcg || pc.use_y;
    const bool lp = K == kPcJacobiPcg && pc.add_p;
    const double alpha = pc.alpha;
    auto load = [&](long long t) {
      RawPc q{};
      if (ly) q.y = yw[t];
      if (lp) q.p = pw[t];
      if (X3 != nullptr) q.x3 = X3[t];
      return q;
    };
    auto value = [&](const RawPc& q) {
      double r = ly ? (double)q.y : 0.0;
      if (lp) r += alpha * (double)q.p;
      if (X3 != nullptr) r += c3 * q.x3;
      return r;
    };
    stencil_march<double>(g, sg, bk.id, stencil_in(load, value), sink);
  } else if constexpr (K == kPcJacobiGmres) {
    // FP32 inner GMRES output with at most kGmRaw columns (checked by the
    // host); a convective operator's velocities are issued at the start of
    // their plane step (the registers leave no room to load them a step ahead)
    if (g.vel != nullptr) stencil_march<double, 2>(g, sg, bk.id, gm_raw_in(pc, X3, c3), sink);
    else stencil_march<double>(g, sg, bk.id, gm_raw_in(pc, X3, c3), sink);
  } else {
    bool done = false;
    if constexpr (GM) {
      if (gm_raw_ok(pc)) {
        stencil_march<double>(g, sg, bk.id, gm_raw_in(pc, X3, c3), sink);
        done = true;
      }
    }
    if (!done) {
      const auto in = stencil_in([&](long long t) {
        double v = pc.at<K, F32>(t);
        if (X3 != nullptr) v += c3 * X3[t];
        return v;
      });
      stencil_march<double>(g, sg, bk.id, in, sink);
    }
  }
  if (dots) block_partials<2>(acc, 2, part, sg.blocks(), bk.id);
}
// Every output kind in one body, for the persistent kernel (whose members'
// kinds are NONE, JACOBI or block PCG): the two inner-CG forms have their own
// branches, the others decide at run time.  GM: the run-time branch also
// carries the FP32 inner-GMRES load-ahead path (more registers).
template <bool GM = false>
__device__ __forceinline__ void apply_pc_out_body(Blk bk, Grid g, StencilGeom sg, PcOutDesc pd, const double* X3,
                                                  double c3, double* __restrict__ O, double* __restrict__ Nout,
                                                  int dots, const double* __restrict__ R, double* part,
                                                  SolveState* st) {
  if (!wg_running(st)) return;
  if (pd.kind == kPcBlockPcg) {
    if (pd.fp32) apply_pc_out_t<kPcBlockPcg, 1>(bk, g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
    else apply_pc_out_t<kPcBlockPcg, 0>(bk, g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
  } else if (pd.kind == kPcJacobiPcg) {
    if (pd.fp32) apply_pc_out_t<kPcJacobiPcg, 1>(bk, g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
    else apply_pc_out_t<kPcJacobiPcg, 0>(bk, g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
  } else {
    apply_pc_out_t<-1, 0, GM>(bk, g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
  }
}
// The single-system kernel: one instantiation per output kind and storage
// (the host picks it from the descriptor), so each carries only its own
// registers.
template <int K, int F32>
__global__ void __launch_bounds__(kBlock)
k_apply_pc_out(Grid g, StencilGeom sg, PcOutDesc pd, const double* X3, double c3,
               double* __restrict__ O, double* __restrict__ Nout,
               int dots, const double* __restrict__ R, double* part, SolveState* st) {
  if (!wg_running(st)) return;
  apply_pc_out_t<K, F32, true>(this_blk(), g, sg, pd, X3, c3, O, Nout, dots, R, part, st);
}

// True-residual verdict after a recurred convergence: kDone or kGap.  part
// holds the partials of ||b - A x||^2; part_nat (natural-norm test) those of
// the true residual's gamma, <B(r), r> or <r, A B(r)>, which then decides
// against the natural tolerance (section 5: other norms confirm it).
__global__ void __launch_bounds__(kBlock)
k_true_check(const double* part, int P, const double* part_nat, int Pn, SolveState* st) {
  const double rr = block_sum_column(part, P, 0);
  const double gg = part_nat != nullptr ? block_sum_column(part_nat, Pn, 0) : 0.0;
  if (threadIdx.x == 0) {
    const double res = sqrt(rr);
    st->true_res = res;
    // before the first start-up's natural norm exists (x0 met the 2-norm
    // tolerance at once) the 2-norm decides
    const bool nat = part_nat != nullptr && st->nat_started;
    const bool ok = nat ? sqrt(fabs(gg)) <= st->ntol : res <= st->tol;
    st->status = ok ? kDone : kGap;
  }
}

// The natural-norm check applies B to the true residual: its kernels run only
// while the status is kRunning, so the check reopens a recurred convergence.
__global__ void k_check_open(SolveState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && st->status == kConverged) st->status = kRunning;
}

// ||b - A x|| at exit, reported only (the status is left as it is).
__global__ void __launch_bounds__(kBlock)
k_true_report(const double* part, int P, SolveState* st) {
  const double rr = block_sum_column(part, P, 0);
  if (threadIdx.x == 0) st->true_res = sqrt(rr);
}

// ---------------------------------------------------------------------------
// PIPEFCG
// ---------------------------------------------------------------------------
// Start-up scalars: history[0], the test on ||r_0||, eta_0 = delta_0, alpha_0.
__global__ void __launch_bounds__(kBlock)
k_pipefcg_init_scalars(const double* part_r, int P_r, const double* part_ud, int P_ud,
                       SolveState* st, double* hist) {
  if (!wg_running(st)) return;
  const double rr = block_sum_column(part_r, P_r, 0);
  const double gamma = block_sum_column(part_ud, P_ud, 0);
  const double delta = block_sum_column(part_ud, P_ud, 1);
  if (threadIdx.x != 0) return;
  const double res = sqrt(rr);
  if (!st->hist_started) { hist[0] = res; log_time(st, 0); st->hist_started = 1; }
  if (!isfinite(res)) { st->status = kNonfinite; return; }
  if (res <= st->tol) { st->status = kConverged; return; }
  natural_start(st, gamma);
  if (!(delta > 0.0) || !isfinite(delta)) { st->status = kBreakdown0; return; }
  st->eta_ring[0] = delta;
  st->alpha = gamma / delta;
  st->j = 0;
  st->nu = 0;
  if (st->it >= st->maxit) st->status = kMaxit;
}

// Two consecutive doubles per lane: one 16-byte access (the scalar tail of
// an odd N reads/writes only .x).  NT: nontemporal accesses, for solves whose
// vectors are far larger than the caches (SolveState::nt; measured on the
// PIPEFCG update at 256^3: 3.66 -> 3.46 ms); small systems keep ordinary
// accesses, whose data the L2 and the Infinity Cache hold between kernels.
typedef double pfk_d2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ double2 ld2(const double* p, long long e, bool full) {
  if constexpr (NT) {
    if (full) {
      const pfk_d2v v = __builtin_nontemporal_load(reinterpret_cast<const pfk_d2v*>(p + e));
      return make_double2(v.x, v.y);
    }
    return make_double2(__builtin_nontemporal_load(p + e), 0.0);
  } else {
    if (full) return *reinterpret_cast<const double2*>(p + e);
    return make_double2(p[e], 0.0);
  }
}
template <bool NT>
__device__ __forceinline__ void st2(double* p, long long e, double2 v, bool full) {
  if constexpr (NT) {
    if (full) {
      pfk_d2v t;
      t.x = v.x;
      t.y = v.y;
      __builtin_nontemporal_store(t, reinterpret_cast<pfk_d2v*>(p + e));
    } else {
      __builtin_nontemporal_store(v.x, p + e);
    }
  } else {
    if (full) *reinterpret_cast<double2*>(p + e) = v;
    else p[e] = v.x;
  }
}

// One fused pass for direction j (= st->j):
//   p_j = u_j + sum beta p_d,  s_j = w_j + sum beta s_d,
//   q_j = m_j + sum beta q_d,  z_j = n_j + sum beta z_d      (written to slot j)
//   x += alpha p_j, r -= alpha s_j, u -= alpha q_j, w -= alpha z_j
// and the single reduction of iteration j+1 on the updated vectors:
//   gamma = <u,r>, delta = <u,w>, rho = <r,r>, <u, s_d> for d in window(j+1)
// (PIPEFCG), or with w in place of u (red_w: PIPEGCR_w, Alg. 12, whose
// vectors and windows are PIPEFCG's with w recurred: gamma = <r,w>,
// delta = <w,w>, <w, s_d>).
// The window dots reuse the s_d loads of the MAXPY.  Each lane owns two
// consecutive nodes (16-byte accesses); the per-direction dot is summed over
// the wave at once and accumulated in LDS, so the register footprint does not
// grow with the window.  Vectors must be 16-byte aligned.
template <bool NT>
__device__ __forceinline__ void pipefcg_update_body_t(Blk bk, long long N, Window P, Window S, Window Q, Window Z,
                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ u,
                 double* __restrict__ w, const double* __restrict__ m, const double* __restrict__ n,
                 double* part, const SolveState* st, int red_w) {
  if (!wg_running(st)) return;
  __shared__ double s_beta[kNuMax];
  __shared__ long long s_off[kNuMax];
  __shared__ double s_dot[kWaves][kNuMax + 4];
  const int j = st->j;
  const int numax = st->nu_max;
  const int nu = trunc_nu(st->trunc, j, numax);         // window of this update
  const int nu1 = trunc_nu(st->trunc, j + 1, numax);    // window of the next reduction
  const int shift = 1 + nu - nu1;                       // first window entry the next dots keep
  const double alpha = st->alpha;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < nu; t += kBlock) {
    s_beta[t] = st->beta[t];
    s_off[t] = (long long)((j - nu + t) % numax) * P.ld;
  }
  for (int t = threadIdx.x; t < kWaves * (kNuMax + 4); t += kBlock) (&s_dot[0][0])[t] = 0.0;
  __syncthreads();
  const long long ns = (long long)(j % numax) * P.ld;
  double gam = 0.0, del = 0.0, rho = 0.0, dnew = 0.0;
  const long long npair = (N + 1) / 2;
  // the trip count is uniform per wave (the in-loop wave sums need every lane);
  // lanes past the end compute on element 0 and contribute nothing
  for (long long qw = bk.gtid() - lane; qw < npair; qw += bk.gstride()) {
    const bool act = qw + lane < npair;
    const long long e = act ? 2 * (qw + lane) : 0;
    const bool full = act && e + 1 < N;
    const double2 u0 = ld2<NT>(u, e, full), w0 = ld2<NT>(w, e, full);
    double2 p = u0, q = ld2<NT>(m, e, full), z = ld2<NT>(n, e, full);
#pragma unroll 4
    for (int t = 0; t < nu; ++t) {
      const double b = s_beta[t];
      const long long o = s_off[t] + e;
      const double2 pv = ld2<NT>(P.base, o, full), qv = ld2<NT>(Q.base, o, full), zv = ld2<NT>(Z.base, o, full);
      p.x += b * pv.x; p.y += b * pv.y;
      q.x += b * qv.x; q.y += b * qv.y;
      z.x += b * zv.x; z.y += b * zv.y;
    }
    const double2 un = make_double2(u0.x - alpha * q.x, u0.y - alpha * q.y);
    const double2 wn = make_double2(w0.x - alpha * z.x, w0.y - alpha * z.y);
    double2 a = red_w ? wn : un;                 // the reduction's first operand
    if (!act) a = make_double2(0.0, 0.0);
    double2 sv = w0;
#pragma unroll 4
    for (int t = 0; t < nu; ++t) {
      const double b = s_beta[t];
      const double2 sd = ld2<NT>(S.base, s_off[t] + e, full);
      sv.x += b * sd.x; sv.y += b * sd.y;
      if (t >= shift) {
        const double d = wave_sum(a.x * sd.x + a.y * sd.y);
        if (lane == 0) s_dot[wid][t - shift] += d;
      }
    }
    if (!act) continue;
    const double2 r0 = ld2<NT>(r, e, full);
    const double2 rn = make_double2(r0.x - alpha * sv.x, r0.y - alpha * sv.y);
    double2 x0 = ld2<NT>(x, e, full);
    x0.x += alpha * p.x; x0.y += alpha * p.y;
    st2<NT>(x, e, x0, full);
    st2<NT>(P.base, ns + e, p, full);
    st2<NT>(S.base, ns + e, sv, full);
    st2<NT>(Q.base, ns + e, q, full);
    st2<NT>(Z.base, ns + e, z, full);
    st2<NT>(u, e, un, full);
    st2<NT>(w, e, wn, full);
    st2<NT>(r, e, rn, full);
    gam += a.x * rn.x + a.y * rn.y;
    del += a.x * wn.x + a.y * wn.y;
    rho += rn.x * rn.x + rn.y * rn.y;
    dnew += a.x * sv.x + a.y * sv.y;
  }
  // columns: gamma, delta, rho, then <u, s_d> for d = j+1-nu1 .. j (the last is s_j)
  const int ncol = 3 + nu1;
  {
    const double a0 = wave_sum(gam), a1 = wave_sum(del), a2 = wave_sum(rho), a3 = wave_sum(dnew);
    if (lane == 0) {
      s_dot[wid][kNuMax] = a0;
      s_dot[wid][kNuMax + 1] = a1;
      s_dot[wid][kNuMax + 2] = a2;
      s_dot[wid][nu1 - 1] = a3;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += kBlock) {
    const int src = c < 3 ? kNuMax + c : c - 3;
    double acc = 0.0;
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) acc += s_dot[wv][src];
    part[(long long)c * bk.n + bk.id] = acc;
  }
}
__device__ __forceinline__ void pipefcg_update_body(Blk bk, long long N, Window P, Window S, Window Q, Window Z,
                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ u,
                 double* __restrict__ w, const double* __restrict__ m, const double* __restrict__ n,
                 double* part, const SolveState* st, int red_w) {
  if (st->nt) pipefcg_update_body_t<true>(bk, N, P, S, Q, Z, x, r, u, w, m, n, part, st, red_w);
  else pipefcg_update_body_t<false>(bk, N, P, S, Q, Z, x, r, u, w, m, n, part, st, red_w);
}
__global__ void __launch_bounds__(kBlock)
k_pipefcg_update(long long N, Window P, Window S, Window Q, Window Z,
                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ u,
                 double* __restrict__ w, const double* __restrict__ m, const double* __restrict__ n,
                 double* part, const SolveState* st, int red_w) {
  pipefcg_update_body(this_blk(), N, P, S, Q, Z, x, r, u, w, m, n, part, st, red_w);
}

// Scalars of iteration j+1 from the fused reduction: iteration count,
// history, convergence test, beta_{j+1,d} = -<u,s_d>/eta_d,
// eta_{j+1} = delta - sum beta^2 eta_d (breakdown if not positive), alpha.
__device__ __forceinline__ void pipefcg_scalars_body(Blk bk, const double* part, int P, SolveState* st, double* hist) {
  __shared__ double col[kNuMax + 3];
  if (!wg_running(st)) return;
  const int j1 = st->j + 1;
  const int nu1 = trunc_nu(st->trunc, j1, st->nu_max);
  block_sum_columns(part, P, 3 + nu1, col);
  if (threadIdx.x != 0) return;
  const int it = st->it + 1;
  st->it = it;
  st->j = j1;
  const double res = sqrt(col[2]);
  hist[it] = res;
  log_time(st, it);
  const double nat = natural_log(st, it, col[0]);
  if (!isfinite(res)) { st->status = kNonfinite; return; }
  if (converged_test(st, res, nat)) { st->status = kConverged; return; }
  if (stalled(st, hist, it, j1, res)) { st->status = kGap; return; }
  const int numax = st->nu_max;
  double eta = col[1];
  for (int t = 0; t < nu1; ++t) {
    const int d = j1 - nu1 + t;
    const double ed = st->eta_ring[d % numax];
    const double b = -col[3 + t] / ed;
    st->beta[t] = b;
    eta -= b * b * ed;
  }
  st->nu = nu1;
  st->eta_new = eta;
  st->gamma = col[0];
  const bool forced = (st->force_it == it);
  if (forced) st->force_it = -1;
  if (forced || !(eta > 0.0) || !isfinite(eta)) { st->status = kBreakdown; return; }
  st->eta_ring[j1 % numax] = eta;
  st->alpha = col[0] / eta;
  if (it >= st->maxit) st->status = kMaxit;
}
__global__ void __launch_bounds__(kBlock)
k_pipefcg_scalars(const double* part, int P, SolveState* st, double* hist) {
  pipefcg_scalars_body(this_blk(), part, P, st, hist);
}

// ---------------------------------------------------------------------------
// FCG and GCR (two blocking reductions per iteration)
// ---------------------------------------------------------------------------
// x += alpha p_j, r -= alpha s_j for the newest direction j = st->j.
__device__ __forceinline__ void fcg_xr_body(Blk bk, long long N, Window P, Window S, double* __restrict__ x, double* __restrict__ r,
         const SolveState* st) {
  if (!wg_running(st)) return;
  const int slot = st->j % st->nu_max;
  const double alpha = st->alpha;
  const double* p = P.slot(slot);
  const double* s = S.slot(slot);
  for (long long e = bk.gtid(); e < N; e += bk.gstride()) {
    x[e] += alpha * p[e];
    r[e] -= alpha * s[e];
  }
}
__global__ void __launch_bounds__(kBlock)
k_fcg_xr(long long N, Window P, Window S, double* __restrict__ x, double* __restrict__ r,
         const SolveState* st) {
  fcg_xr_body(this_blk(), N, P, S, x, r, st);
}

// The multi-dot of one vector V against R, itself and the window:
// columns <V,R>, <V,V>, <R,R>, then <V, S_d> for d in window(j+1), j = st->j
// (an empty window with `init`).  V is read from Vin, or formed from the
// preconditioner's output (from_pc) and written to Vout.
//   FCG:     V = u = B(r), R = r  (gamma = <u,r>, the test on <r,r>, <u,s_d>)
//   GCR:     V = t = A u,  R = r  (the test on <r,r>, <t,s_d>)
//   PIPEGCR: V = w = A u,  R = r  (gamma, delta, rho, <w,s_d>: its single reduction)
template <bool NT>
__device__ __forceinline__ void multidot_body_t(Blk bk, long long N, int init, int from_pc, PcOutDesc pd, const double* __restrict__ Vin,
           double* __restrict__ Vout, const double* __restrict__ R, Window S, double* part, SolveState* st) {
  if (!wg_running(st)) return;
  PcOut pc{};
  if (from_pc) pc = make_pc_out(pd, &st->pc);
  __shared__ long long s_off[kNuMax];
  __shared__ double s_dot[kWaves][kNuMax + 3];
  const int j1 = st->j + 1;
  const int numax = st->nu_max;
  const int nu = init ? 0 : trunc_nu(st->trunc, j1, numax);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < nu; t += kBlock) s_off[t] = (long long)((j1 - nu + t) % numax) * S.ld;
  for (int t = threadIdx.x; t < kWaves * (kNuMax + 3); t += kBlock) (&s_dot[0][0])[t] = 0.0;
  __syncthreads();
  // Windows of up to kDotRegs directions (the configurations' 20 and 30)
  // keep one accumulator per direction in registers and sum over the wave
  // once at the end; longer windows sum every direction's products over the
  // wave inside the loop.
  constexpr int kDotRegs = 32;
  const bool regs = nu <= kDotRegs;
  double acc[kDotRegs];
#pragma unroll
  for (int t = 0; t < kDotRegs; ++t) acc[t] = 0.0;
  double vr = 0.0, vv = 0.0, rr = 0.0;
  const long long npair = (N + 1) / 2;
  // wave-uniform trip count (the long-window path sums over the wave inside);
  // lanes past the end use element 0 and contribute nothing.  Each lane owns
  // two consecutive nodes (16-byte accesses).
  for (long long qw = bk.gtid() - lane; qw < npair; qw += bk.gstride()) {
    const bool act = qw + lane < npair;
    const long long e = act ? 2 * (qw + lane) : 0;
    const bool full = act && e + 1 < N;
    double2 v = make_double2(0.0, 0.0);
    if (from_pc) {
      if (act) {
        v.x = pc(e);
        if (full) v.y = pc(e + 1);
        st2<NT>(Vout, e, v, full);
      }
    } else if (act) {
      v = ld2<NT>(Vin, e, full);
    }
    const double2 r = act ? ld2<NT>(R, e, full) : make_double2(0.0, 0.0);
    vr += v.x * r.x + v.y * r.y;
    vv += v.x * v.x + v.y * v.y;
    rr += r.x * r.x + r.y * r.y;
    if (regs) {
      // eight directions at a time: their loads in flight together, the
      // compiler kept from hoisting the next group's (registers)
#pragma unroll
      for (int c = 0; c < kDotRegs; c += 8) {
        if (c < nu) {
#pragma unroll
          for (int t = c; t < c + 8; ++t) {
            if (t < nu) {
              const double2 sd = ld2<NT>(S.base, s_off[t] + e, full);
              acc[t] += v.x * sd.x + v.y * sd.y;
            }
          }
        }
        asm volatile("" ::: "memory");
      }
    } else {
      for (int t = 0; t < nu; ++t) {
        const double2 sd = ld2<NT>(S.base, s_off[t] + e, full);
        const double d = wave_sum(v.x * sd.x + v.y * sd.y);
        if (lane == 0) s_dot[wid][3 + t] += d;
      }
    }
  }
  if (regs) {
#pragma unroll
    for (int t = 0; t < kDotRegs; ++t) {
      if (t < nu) {
        const double d = wave_sum(acc[t]);
        if (lane == 0) s_dot[wid][3 + t] = d;
      }
    }
  }
  {
    const double a0 = wave_sum(vr), a1 = wave_sum(vv), a2 = wave_sum(rr);
    if (lane == 0) { s_dot[wid][0] = a0; s_dot[wid][1] = a1; s_dot[wid][2] = a2; }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < 3 + nu; c += kBlock) {
    double a = 0.0;
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) a += s_dot[wv][c];
    part[(long long)c * bk.n + bk.id] = a;
  }
}
__device__ __forceinline__ void multidot_body(Blk bk, long long N, int init, int from_pc, PcOutDesc pd, const double* __restrict__ Vin,
           double* __restrict__ Vout, const double* __restrict__ R, Window S, double* part, SolveState* st) {
  if (st->nt) multidot_body_t<true>(bk, N, init, from_pc, pd, Vin, Vout, R, S, part, st);
  else multidot_body_t<false>(bk, N, init, from_pc, pd, Vin, Vout, R, S, part, st);
}
__global__ void __launch_bounds__(kBlock)
k_multidot(long long N, int init, int from_pc, PcOutDesc pd, const double* __restrict__ Vin,
           double* __restrict__ Vout, const double* __restrict__ R, Window S, double* part, SolveState* st) {
  multidot_body(this_blk(), N, init, from_pc, pd, Vin, Vout, R, S, part, st);
}

// First-reduction scalars of FCG/GCR from k_multidot's columns: the
// iteration count, history and test on ||r||, beta_d = -<V,s_d>/eta_d, and
// (FCG) gamma = <u, r>.  With `init` only j = 0 and gamma are set.
__device__ __forceinline__ void cg_scalars1_body(Blk bk, int init, const double* part, int P, SolveState* st, double* hist) {
  __shared__ double col[kNuMax + 3];
  if (!wg_running(st)) return;
  const int j1 = init ? 0 : st->j + 1;
  const int nu = init ? 0 : trunc_nu(st->trunc, j1, st->nu_max);
  block_sum_columns(part, P, 3 + nu, col);
  if (threadIdx.x != 0) return;
  st->gamma = col[0];
  st->nu = nu;
  st->j = j1;
  if (init) {
    natural_start(st, col[0]);
    return;
  }
  const int it = st->it + 1;
  st->it = it;
  const double res = sqrt(col[2]);
  hist[it] = res;
  log_time(st, it);
  const double nat = natural_log(st, it, col[0]);
  if (!isfinite(res)) { st->status = kNonfinite; return; }
  if (converged_test(st, res, nat)) { st->status = kConverged; return; }
  if (stalled(st, hist, it, j1, res)) { st->status = kGap; return; }
  const int numax = st->nu_max;
  for (int t = 0; t < nu; ++t) {
    const int d = j1 - nu + t;
    st->beta[t] = -col[3 + t] / st->eta_ring[d % numax];
  }
}
__global__ void __launch_bounds__(kBlock)
k_cg_scalars1(int init, const double* part, int P, SolveState* st, double* hist) {
  cg_scalars1_body(this_blk(), init, part, P, st, hist);
}

// p_j = u + sum beta p_d into slot j (FCG).
template <bool NT>
__device__ __forceinline__ void fcg_maxpy_body_t(Blk bk, long long N, Window P, const double* __restrict__ u, const SolveState* st) {
  if (!wg_running(st)) return;
  __shared__ double s_beta[kNuMax];
  __shared__ long long s_off[kNuMax];
  const int j = st->j, nu = st->nu, numax = st->nu_max;
  for (int t = threadIdx.x; t < nu; t += kBlock) {
    s_beta[t] = st->beta[t];
    s_off[t] = (long long)((j - nu + t) % numax) * P.ld;
  }
  __syncthreads();
  double* pn = P.slot(j % numax);
  const long long npair = (N + 1) / 2;
  for (long long qi = bk.gtid(); qi < npair; qi += bk.gstride()) {
    const long long e = 2 * qi;
    const bool full = e + 1 < N;
    double2 p = ld2<NT>(u, e, full);
    int t = 0;
    for (; t + 4 <= nu; t += 4) {
      double2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = ld2<NT>(P.base, s_off[t + q] + e, full);
#pragma unroll
      for (int q = 0; q < 4; ++q) { p.x += s_beta[t + q] * v[q].x; p.y += s_beta[t + q] * v[q].y; }
    }
    for (; t < nu; ++t) {
      const double2 v = ld2<NT>(P.base, s_off[t] + e, full);
      p.x += s_beta[t] * v.x; p.y += s_beta[t] * v.y;
    }
    st2<NT>(pn, e, p, full);
  }
}
__device__ __forceinline__ void fcg_maxpy_body(Blk bk, long long N, Window P, const double* __restrict__ u, const SolveState* st) {
  if (st->nt) fcg_maxpy_body_t<true>(bk, N, P, u, st);
  else fcg_maxpy_body_t<false>(bk, N, P, u, st);
}
__global__ void __launch_bounds__(kBlock)
k_fcg_maxpy(long long N, Window P, const double* __restrict__ u, const SolveState* st) {
  fcg_maxpy_body(this_blk(), N, P, u, st);
}

// GCR: p_j = u + sum beta p_d, s_j = t + sum beta s_d into slot j, partials
// <r, s_j>, <s_j, s_j> (gamma and eta of the second reduction).
template <bool NT>
__device__ __forceinline__ void gcr_maxpy_t(long long N, Window P, Window S, const double* __restrict__ u,
                                            const double* __restrict__ t_, const double* __restrict__ r,
                                            double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  __shared__ double s_beta[kNuMax];
  __shared__ long long s_off[kNuMax];
  const int j = st->j, nu = st->nu, numax = st->nu_max;
  for (int t = threadIdx.x; t < nu; t += kBlock) {
    s_beta[t] = st->beta[t];
    s_off[t] = (long long)((j - nu + t) % numax) * P.ld;
  }
  __syncthreads();
  const long long ns = (long long)(j % numax) * P.ld;
  double acc[2] = {0.0, 0.0};
  const long long npair = (N + 1) / 2;
  for (long long qi = gtid(); qi < npair; qi += gstride()) {
    const long long e = 2 * qi;
    const bool full = e + 1 < N;
    double2 p = ld2<NT>(u, e, full), s = ld2<NT>(t_, e, full);
    for (int t = 0; t < nu; ++t) {
      const double b = s_beta[t];
      const double2 pv = ld2<NT>(P.base, s_off[t] + e, full), sv = ld2<NT>(S.base, s_off[t] + e, full);
      p.x += b * pv.x; p.y += b * pv.y;
      s.x += b * sv.x; s.y += b * sv.y;
    }
    st2<NT>(P.base, ns + e, p, full);
    st2<NT>(S.base, ns + e, s, full);
    const double2 rv = ld2<NT>(r, e, full);
    acc[0] += rv.x * s.x + rv.y * s.y;
    acc[1] += s.x * s.x + s.y * s.y;
  }
  block_partials<2>(acc, 2, part, gridDim.x);
}
__global__ void __launch_bounds__(kBlock)
k_gcr_maxpy(long long N, Window P, Window S, const double* __restrict__ u, const double* __restrict__ t_,
            const double* __restrict__ r, double* part, const SolveState* st) {
  if (st->nt) gcr_maxpy_t<true>(N, P, S, u, t_, r, part, st);
  else gcr_maxpy_t<false>(N, P, S, u, t_, r, part, st);
}

// s_j = A p_j, partial eta_j = <p_j, s_j> (FCG).
__device__ __forceinline__ void fcg_apply_body(Blk bk, Grid g, StencilGeom sg, Window P, Window S, double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  const int slot = st->j % st->nu_max;
  const double* p = P.slot(slot);
  double* s = S.slot(slot);
  double acc[1] = {0.0};
  const auto in = stencil_in([&](long long t) { return p[t]; });
  auto sink = [&](long long idx, double pc, double sv) {
    s[idx] = sv;
    acc[0] += pc * sv;
  };
  stencil_march<double>(g, sg, bk.id, in, sink);
  block_partials<1>(acc, 1, part, sg.blocks(), bk.id);
}
__global__ void __launch_bounds__(kBlock)
k_fcg_apply(Grid g, StencilGeom sg, Window P, Window S, double* part, const SolveState* st) {
  fcg_apply_body(this_blk(), g, sg, P, S, part, st);
}

// Second-reduction scalars: eta_j (FCG: <p,s>; GCR: <s,s> with gamma = <r,s>),
// breakdown check, alpha_j.
__device__ __forceinline__ void cg_scalars2_body(Blk bk, int gcr, int init, const double* part, int P, SolveState* st) {
  if (!wg_running(st)) return;
  const double c0 = block_sum_column(part, P, 0);
  const double c1 = gcr ? block_sum_column(part, P, 1) : 0.0;
  if (threadIdx.x != 0) return;
  const double eta = gcr ? c1 : c0;
  if (gcr) st->gamma = c0;
  const int j = st->j;
  if (!init) {
    const bool forced = (st->force_it == st->it);
    if (forced) st->force_it = -1;
    if (forced || !(eta > 0.0) || !isfinite(eta)) { st->status = kBreakdown; return; }
  } else if (!(eta > 0.0) || !isfinite(eta)) {
    st->status = kBreakdown0;
    return;
  }
  st->eta_ring[j % st->nu_max] = eta;
  st->alpha = st->gamma / eta;
  if (st->it >= st->maxit) st->status = kMaxit;
}
__global__ void __launch_bounds__(kBlock)
k_cg_scalars2(int gcr, int init, const double* part, int P, SolveState* st) {
  cg_scalars2_body(this_blk(), gcr, init, part, P, st);
}

// Start-up test on ||r_0|| (history[0]).
__global__ void __launch_bounds__(kBlock)
k_init_test(const double* part, int P, SolveState* st, double* hist) {
  if (!wg_running(st)) return;
  const double rr = block_sum_column(part, P, 0);
  if (threadIdx.x != 0) return;
  const double res = sqrt(rr);
  if (!st->hist_started) { hist[0] = res; log_time(st, 0); st->hist_started = 1; }
  if (!isfinite(res)) { st->status = kNonfinite; return; }
  if (res <= st->tol) st->status = kConverged;
  else if (st->it >= st->maxit) st->status = kMaxit;
}

// ---------------------------------------------------------------------------
// PIPEGCR (Alg. 11)
// ---------------------------------------------------------------------------
// Start-up scalars from the start-up multi-dot (V = w_0 = s_0 = A u_0,
// R = r_0): gamma_0 = <r_0, s_0>, eta_0 = <s_0, s_0>, alpha_0.
__global__ void __launch_bounds__(kBlock)
k_pipegcr_init_scalars(const double* part, int P, SolveState* st) {
  if (!wg_running(st)) return;
  const double gamma = block_sum_column(part, P, 0);
  const double eta = block_sum_column(part, P, 1);
  if (threadIdx.x != 0) return;
  natural_start(st, gamma);
  if (!(eta > 0.0) || !isfinite(eta)) { st->status = kBreakdown0; return; }
  st->eta_ring[0] = eta;
  st->alpha = gamma / eta;
  st->j = 0;
  st->nu = 0;
  if (st->it >= st->maxit) st->status = kMaxit;
}

// Direction j (= st->j):  p_j = u + sum beta p_d,  s_j = w + sum beta s_d,
// q_j = m + sum beta q_d into slot j, then x += alpha p_j, r -= alpha s_j,
// u -= alpha q_j.  m = u + B(w - r) is evaluated from the inner solve's
// output; for the first direction after a (re)start it is q_0's B(s_0).
// As in PIPEFCG's update: two consecutive nodes per lane (16-byte accesses,
// nontemporal for large solves), the three windows' loads of a direction
// taken together (twelve in flight with the loop unrolled by four), and an
// FP32 inner GMRES output read two nodes per 8-byte load.  Each node's
// arithmetic is the one-node form's, in the same order.
template <bool NT>
__device__ __forceinline__ void pipegcr_update_body_t(Blk bk, long long N, Window P, Window S, Window Q,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ u, const double* __restrict__ w,
                                                      PcOutDesc pd, SolveState* st) {
  __shared__ double s_beta[kNuMax];
  __shared__ long long s_off[kNuMax];
  const int j = st->j;
  const int numax = st->nu_max;
  const int nu = trunc_nu(st->trunc, j, numax);
  const double alpha = st->alpha;
  const bool first = (j == 0);
  if (first) pd.X2 = nullptr;                  // q_0 = B(s_0): the start-up input was w alone
  const PcOut pc = make_pc_out(pd, &st->pc);
  const double cu = first ? 0.0 : 1.0;
  for (int t = threadIdx.x; t < nu; t += kBlock) {
    s_beta[t] = st->beta[t];
    s_off[t] = (long long)((j - nu + t) % numax) * P.ld;
  }
  __syncthreads();
  const long long ns = (long long)(j % numax) * P.ld;
  const bool gm2 = gm_raw_ok(pc);
  const float* gmV = static_cast<const float*>(pc.vbase);
  const float* gmD = static_cast<const float*>(pc.dinv_in);
  const long long npair = (N + 1) / 2;
  for (long long qp = bk.gtid(); qp < npair; qp += bk.gstride()) {
    const long long e = 2 * qp;
    const bool full = e + 1 < N;
    const double2 u0 = ld2<NT>(u, e, full), w0 = ld2<NT>(w, e, full);
    double2 bv;
    if (gm2 && full) {
      float2 vq[kGmRaw];
#pragma unroll
      for (int q = 0; q < kGmRaw; ++q)
        vq[q] = q < pc.nv ? *reinterpret_cast<const float2*>(gmV + (long long)q * pc.ldv + e) : make_float2(0.f, 0.f);
      const float2 dv = *reinterpret_cast<const float2*>(gmD + e);
      double r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int q = 0; q < kGmRaw; ++q) {
        if (q < pc.nv) {
          r0 += pc.cf[q] * (double)vq[q].x;
          r1 += pc.cf[q] * (double)vq[q].y;
        }
      }
      bv = make_double2((double)dv.x * r0, (double)dv.y * r1);
    } else {
      bv = make_double2(pc(e), full ? pc(e + 1) : 0.0);
    }
    double2 p = u0, sv = w0;
    double2 q = make_double2(cu * u0.x + bv.x, cu * u0.y + bv.y);
#pragma unroll 4
    for (int t = 0; t < nu; ++t) {
      const double b = s_beta[t];
      const long long o = s_off[t] + e;
      const double2 pv = ld2<NT>(P.base, o, full), svv = ld2<NT>(S.base, o, full), qv = ld2<NT>(Q.base, o, full);
      p.x += b * pv.x; p.y += b * pv.y;
      sv.x += b * svv.x; sv.y += b * svv.y;
      q.x += b * qv.x; q.y += b * qv.y;
    }
    st2<NT>(P.base, ns + e, p, full);
    st2<NT>(S.base, ns + e, sv, full);
    st2<NT>(Q.base, ns + e, q, full);
    double2 x0 = ld2<NT>(x, e, full), r0v = ld2<NT>(r, e, full);
    x0.x += alpha * p.x; x0.y += alpha * p.y;
    r0v.x -= alpha * sv.x; r0v.y -= alpha * sv.y;
    st2<NT>(x, e, x0, full);
    st2<NT>(r, e, r0v, full);
    st2<NT>(u, e, make_double2(u0.x - alpha * q.x, u0.y - alpha * q.y), full);
  }
}
__global__ void __launch_bounds__(kBlock)
k_pipegcr_update(long long N, Window P, Window S, Window Q, double* __restrict__ x, double* __restrict__ r,
                 double* __restrict__ u, const double* __restrict__ w, PcOutDesc pd, SolveState* st) {
  if (!wg_running(st)) return;
  if (st->nt) pipegcr_update_body_t<true>(this_blk(), N, P, S, Q, x, r, u, w, pd, st);
  else pipegcr_update_body_t<false>(this_blk(), N, P, S, Q, x, r, u, w, pd, st);
}

}  // namespace pfk
