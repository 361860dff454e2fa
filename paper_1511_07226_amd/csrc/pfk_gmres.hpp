// Outer kernels of the GMRES family: FGMRES (Alg. 13) and PIPEFGMRES
// (Alg. 15), restarted every m columns.
//
// Storage: basis windows P (p_0..p_m), U (the preconditioned vectors u_j or
// u~_j) and, for PIPEFGMRES, ZB (z-bar_j), each column j at slot j.  Column
// slots are taken from the device state (st->col), so one captured graph
// serves every column.  The Hessenberg least squares is solved on the fly by
// Givens rotations in single-workgroup kernels; when a cycle ends (converged,
// happy breakdown, m columns, iteration limit or a PIPEFGMRES norm breakdown)
// the solution coefficients y are stored and x = x0 + U y is applied by
// k_gm_update_x.  That update is idempotent (x0 is saved at the cycle start),
// so replaying it in later enqueued iterations changes nothing.
#pragma once
#include "pfk_cg.hpp"

namespace pfk {

// Rotated Hessenberg R is column-major with kNuMax+1 rows.
constexpr int kRrows = kNuMax + 1;

// Append Hessenberg column c (entries h[0..c], subdiagonal hn): apply the
// previous rotations, form the new one, update g; returns |g[c+1]|, the
// least-squares residual.  Single thread.
__device__ inline double gm_add_column(SolveState* st, int c, const double* h, double hn) {
  double* R = st->R + (long long)c * kRrows;
  for (int i = 0; i <= c; ++i) R[i] = h[i];
  R[c + 1] = hn;
  for (int i = 0; i < c; ++i) {
    const double a = R[i], b = R[i + 1];
    R[i] = st->cs[i] * a + st->sn[i] * b;
    R[i + 1] = -st->sn[i] * a + st->cs[i] * b;
  }
  const double a = R[c], b = R[c + 1];
  const double d = hypot(a, b);
  const double cc = d == 0.0 ? 1.0 : a / d;
  const double ss = d == 0.0 ? 0.0 : b / d;
  st->cs[c] = cc;
  st->sn[c] = ss;
  R[c] = d;
  R[c + 1] = 0.0;
  const double gc = st->g[c];
  st->g[c] = cc * gc;
  st->g[c + 1] = -ss * gc;
  return fabs(st->g[c + 1]);
}

// y = R^-1 g over the first ncol columns; marks the cycle-end update.
__device__ inline void gm_finish_cycle(SolveState* st, int ncol) {
  for (int i = ncol - 1; i >= 0; --i) {
    double acc = st->g[i];
    for (int j = i + 1; j < ncol; ++j) acc -= st->R[(long long)j * kRrows + i] * st->y[j];
    st->y[i] = acc / st->R[(long long)i * kRrows + i];
  }
  st->ycols = ncol;
  st->pend = ncol > 0;
}

// Cycle start after r = b - A x (x0 saved): beta_0, history[0], the test on
// ||r_0||, g = beta_0 e_0, the scale 1/beta_0 of p_0.
__global__ void __launch_bounds__(kBlock)
k_gm_cycle_start(const double* part, int P, SolveState* st, double* hist) {
  if (!wg_running(st)) return;
  const double rr = block_sum_column(part, P, 0);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(rr);
  if (!st->hist_started) { hist[0] = beta; log_time(st, 0); st->hist_started = 1; }
  st->col = 0;
  st->pend = 0;
  st->ycols = 0;
  if (!isfinite(beta)) { st->status = kNonfinite; return; }
  if (beta <= st->tol) { st->status = kConverged; return; }
  st->beta0 = beta;
  st->g[0] = beta;
  st->inv_hn = 1.0 / beta;
  if (st->it >= st->maxit) st->status = kMaxit;
}

// P[col] = src * inv_hn and a copy for the preconditioner's input.  src is
// r (cycle start) or, with from_window, the unnormalised P[col] itself.
__global__ void __launch_bounds__(kBlock)
k_gm_scale(long long N, const double* src, int from_window, Window P, double* __restrict__ vin,
           const SolveState* st) {
  if (!wg_running(st)) return;
  const double sc = st->inv_hn;
  double* dst = P.slot(st->col);
  const double* s = from_window ? dst : src;
  for (long long e = gtid(); e < N; e += gstride()) {
    const double v = s[e] * sc;
    dst[e] = v;
    vin[e] = v;
  }
}

// x = x0 + sum_j y_j U[j] once a cycle has ended (idempotent).
__device__ __forceinline__ void gm_update_x_body(Blk bk, long long N, Window U, const double* __restrict__ x0, double* __restrict__ x, const SolveState* st) {
  if (!st->pend) return;
  __shared__ double s_y[kNuMax];
  const int n = st->ycols;
  for (int t = threadIdx.x; t < n; t += kBlock) s_y[t] = st->y[t];
  __syncthreads();
  for (long long e = bk.gtid(); e < N; e += bk.gstride()) {
    double v = x0[e];
    for (int j = 0; j < n; ++j) v += s_y[j] * U.base[(long long)j * U.ld + e];
    x[e] = v;
  }
}
__global__ void __launch_bounds__(kBlock)
k_gm_update_x(long long N, Window U, const double* __restrict__ x0, double* __restrict__ x, const SolveState* st) {
  gm_update_x_body(this_blk(), N, U, x0, x, st);
}

// ---------------------------------------------------------------------------
// FGMRES
// ---------------------------------------------------------------------------
// u_c = B(p_c) into U[c] and z = A u_c (c = st->col).
__global__ void __launch_bounds__(kBlock)
k_fgm_apply(Grid g, StencilGeom sg, PcOutDesc pd, Window U, double* __restrict__ z, SolveState* st) {
  if (!wg_running(st)) return;
  const PcOut pc = make_pc_out(pd, &st->pc);
  double* uc = U.slot(st->col);
  const auto in = stencil_in([&](long long t) { return pc(t); });
  auto sink = [&](long long idx, double u, double Au) {
    uc[idx] = u;
    z[idx] = Au;
  };
  // loads two plane steps ahead (no occupancy step lost)
  if (gm_raw_ok(pc)) stencil_march<double, false, 2>(g, sg, gm_raw_in(pc, nullptr, 0.0), sink);
  else stencil_march<double, false, 2>(g, sg, in, sink);
}

// First reduction: <p_j, z> for j <= c.
__global__ void __launch_bounds__(kBlock)
k_fgm_dots(long long N, Window P, const double* __restrict__ z, double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  __shared__ double s_dot[kWaves][kNuMax + 1];
  const int nc = st->col + 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < kWaves * (kNuMax + 1); t += kBlock) (&s_dot[0][0])[t] = 0.0;
  __syncthreads();
  const long long step = 2LL * gstride();
  // wave-uniform trip count (wave sums inside); lanes past the end contribute 0
  for (long long w0 = 2LL * blockIdx.x * kBlock + threadIdx.x - lane; w0 < N; w0 += step) {
    const long long e0 = w0 + lane;
    const bool h0 = e0 < N;
    const long long e1 = e0 + kBlock;
    const bool h1 = e1 < N;
    const double z0 = h0 ? z[e0] : 0.0, z1 = h1 ? z[e1] : 0.0;
    for (int j = 0; j < nc; ++j) {
      const double* p = P.base + (long long)j * P.ld;
      const double d = wave_sum((h0 ? z0 * p[e0] : 0.0) + (h1 ? z1 * p[e1] : 0.0));
      if (lane == 0) s_dot[wid][j] += d;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += kBlock) {
    double acc = 0.0;
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) acc += s_dot[wv][c];
    part[(long long)c * gridDim.x + blockIdx.x] = acc;
  }
}

// h_j = sum of column j (single workgroup).
__global__ void __launch_bounds__(kBlock)
k_gm_hbar(const double* part, int P, SolveState* st) {
  __shared__ double col[kNuMax + 1];
  if (!wg_running(st)) return;
  const int nc = st->col + 1;
  block_sum_columns(part, P, nc, col);
  for (int c = threadIdx.x; c < nc; c += kBlock) st->hbar[c] = col[c];
}

// p-bar = z - sum_j h_j p_j into P[c+1] (unnormalised), partial ||p-bar||^2.
__global__ void __launch_bounds__(kBlock)
k_fgm_orth(long long N, Window P, const double* __restrict__ z, double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  __shared__ double s_h[kNuMax + 1];
  const int nc = st->col + 1;
  for (int t = threadIdx.x; t < nc; t += kBlock) s_h[t] = st->hbar[t];
  __syncthreads();
  double* pn = P.slot(nc);
  double acc[1] = {0.0};
  for (long long e = gtid(); e < N; e += gstride()) {
    double v = z[e];
    for (int j = 0; j < nc; ++j) v -= s_h[j] * P.base[(long long)j * P.ld + e];
    pn[e] = v;
    acc[0] += v * v;
  }
  block_partials<1>(acc, 1, part, gridDim.x);
}

// Second reduction: h_{c+1,c} = ||p-bar||, Givens, history, test, cycle end.
__global__ void __launch_bounds__(kBlock)
k_fgm_column(const double* part, int P, SolveState* st, double* hist) {
  if (!wg_running(st)) return;
  const double nn = block_sum_column(part, P, 0);
  if (threadIdx.x != 0) return;
  const int c = st->col;
  const double hn = sqrt(nn);
  if (!isfinite(hn)) { st->status = kNonfinite; return; }
  const double res = gm_add_column(st, c, st->hbar, hn);
  const int it = st->it + 1;
  st->it = it;
  hist[it] = res;
  log_time(st, it);
  st->hn = hn;
  if (res <= st->tol || hn == 0.0) { gm_finish_cycle(st, c + 1); st->status = kConverged; return; }
  if (c + 1 == st->nu_max) { gm_finish_cycle(st, c + 1); st->status = kCycleEnd; return; }
  if (it >= st->maxit) { gm_finish_cycle(st, c + 1); st->status = kMaxit; return; }
  st->inv_hn = 1.0 / hn;
  st->col = c + 1;
}

// ---------------------------------------------------------------------------
// PIPEFGMRES
// ---------------------------------------------------------------------------
// Cycle start: u~_0 = B(p_0) into U[0], zbar_0 = A u~_0 - sigma p_0 into ZB[0]
// and zin; partials <p_0, zbar_0>, <zbar_0, zbar_0> (the first reduction).
__global__ void __launch_bounds__(kBlock)
k_pgm_apply0(Grid g, StencilGeom sg, PcOutDesc pd, Window U, Window P, Window ZB, double* __restrict__ zin,
             double* part, SolveState* st) {
  if (!wg_running(st)) return;
  const PcOut pc = make_pc_out(pd, &st->pc);
  const double sigma = st->sigma;
  double* u0 = U.slot(0);
  const double* p0 = P.slot(0);
  double* z0 = ZB.slot(0);
  double acc[2] = {0.0, 0.0};
  const auto in = stencil_in([&](long long t) { return pc(t); });
  auto sink = [&](long long idx, double u, double Au) {
    const double pv = p0[idx];
    const double zb = Au - sigma * pv;
    u0[idx] = u;
    z0[idx] = zb;
    zin[idx] = zb;
    acc[0] += pv * zb;
    acc[1] += zb * zb;
  };
  if (gm_raw_ok(pc)) stencil_march<double>(g, sg, gm_raw_in(pc, nullptr, 0.0), sink);
  else stencil_march<double>(g, sg, in, sink);
  block_partials<2>(acc, 2, part, sg.blocks());
}

// The single reduction's scalars for column c = st->col: hbar_j = <p_j, zbar_c>,
// t = ||zbar_c||^2 - sum hbar_j^2 (t < 0: norm breakdown -> finish with the
// columns so far and restart), h_{c,c} = hbar_c + sigma, h_{c+1,c} = sqrt(t),
// Givens, history, test, cycle end.
__device__ __forceinline__ void pgm_scalars_body(Blk bk, const double* part, int P, SolveState* st, double* hist) {
  __shared__ double col[kNuMax + 2];
  if (!wg_running(st)) return;
  const int c = st->col;
  block_sum_columns(part, P, c + 2, col);
  if (threadIdx.x != 0) return;
  const double zeta = col[c + 1];
  double t = zeta;
  for (int j = 0; j <= c; ++j) t -= col[j] * col[j];
  const int nxt = st->it + 1;
  const bool forced = (st->force_it == nxt);
  if (forced) st->force_it = -1;
  if (!isfinite(zeta)) { st->status = kNonfinite; return; }
  if (forced || t < 0.0) {
    gm_finish_cycle(st, c);
    st->status = kBreakdown;
    return;
  }
  const double hn = sqrt(t);
  double* h = col;                         // reuse the column buffer for the shifted column
  for (int j = 0; j <= c; ++j) {
    st->hbar[j] = col[j];
    h[j] = col[j];
  }
  h[c] += st->sigma;
  const double res = gm_add_column(st, c, h, hn);
  st->it = nxt;
  hist[nxt] = res;
  log_time(st, nxt);
  st->hn = hn;
  if (res <= st->tol || hn == 0.0) { gm_finish_cycle(st, c + 1); st->status = kConverged; return; }
  if (c + 1 == st->nu_max) { gm_finish_cycle(st, c + 1); st->status = kCycleEnd; return; }
  if (nxt >= st->maxit) { gm_finish_cycle(st, c + 1); st->status = kMaxit; return; }
  st->inv_hn = 1.0 / hn;
  st->col = c + 1;
}
__global__ void __launch_bounds__(kBlock)
k_pgm_scalars(const double* part, int P, SolveState* st, double* hist) {
  pgm_scalars_body(this_blk(), part, P, st, hist);
}

// Column n = st->col (after the scalars of column n-1):
//   p_n   = (zbar_{n-1} - sum_j hbar_j p_j) / h
//   u~_n  = (qbar_{n-1} - sum_j hbar_j u~_j) / h,     qbar = B(zbar) (inner solve output)
//   zbar_n = (wbar_{n-1} - sigma zbar_{n-1} - sum_j hbar_j zbar_j) / h
// into slot n (zbar_n also to zin), and the next single reduction:
// <p_j, zbar_n> for j <= n and ||zbar_n||^2.
// As in PIPEFCG's update, each lane owns two consecutive nodes (16-byte
// accesses).  Two window passes per node pair, each keeping eight loads in
// flight: zbar first (its loop unrolled by eight), then p and u~ together
// (by four), since the dots with p_j need the finished zbar_n and reuse the
// p_j loads.  The inner solve's output is loaded before the zbar pass and
// combined after it, so its loads overlap that pass.  Each vector subtracts
// its terms in order j = 0, 1, ..., as the method writes them.
template <bool NT>
__device__ __forceinline__ void pgm_update_body_t(Blk bk, long long N, Window P, Window U, Window ZB, PcOutDesc pd, const double* __restrict__ wb,
             double* __restrict__ zin, double* part, SolveState* st) {
  if (!wg_running(st)) return;
  const PcOut pc = make_pc_out(pd, &st->pc);
  __shared__ double s_h[kNuMax + 1];
  __shared__ double s_dot[kWaves][kNuMax + 2];
  const int n = st->col;                  // new column; hbar_j for j < n
  const double inv = st->inv_hn;
  const double sigma = st->sigma;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < n; t += kBlock) s_h[t] = st->hbar[t];
  for (int t = threadIdx.x; t < kWaves * (kNuMax + 2); t += kBlock) (&s_dot[0][0])[t] = 0.0;
  __syncthreads();
  const double* zprev = ZB.slot(n - 1);
  double* pn = P.slot(n);
  double* un = U.slot(n);
  double* zn = ZB.slot(n);
  double dp = 0.0, zz = 0.0;
  const bool gm2 = gm_raw_ok(pc);
  const float* gmV = static_cast<const float*>(pc.vbase);
  const float* gmD = static_cast<const float*>(pc.dinv_in);
  const long long npair = (N + 1) / 2;
  // wave-uniform trip count (wave sums inside); lanes past the end use
  // element 0, contribute 0 and store nothing
  for (long long qw = bk.gtid() - lane; qw < npair; qw += bk.gstride()) {
    const bool act = qw + lane < npair;
    const long long e = act ? 2 * (qw + lane) : 0;
    const bool full = act && e + 1 < N;
    const double2 zp = ld2<NT>(zprev, e, full), wv = ld2<NT>(wb, e, full);
    // B(zbar) from an FP32 inner GMRES output, both nodes per 8-byte load
    // (PcOut's arithmetic: dinv * sum cf_q V_q), loads issued here
    const bool gmf = gm2 && full;
    float2 dv = make_float2(0.f, 0.f), vq[kGmRaw];
#pragma unroll
    for (int q = 0; q < kGmRaw; ++q) {
      vq[q] = make_float2(0.f, 0.f);
      if (gmf && q < pc.nv) vq[q] = *reinterpret_cast<const float2*>(gmV + (long long)q * pc.ldv + e);
    }
    if (gmf) dv = *reinterpret_cast<const float2*>(gmD + e);
    double2 z = make_double2(wv.x - sigma * zp.x, wv.y - sigma * zp.y);
#pragma unroll 8
    for (int j = 0; j < n; ++j) {
      const double h = s_h[j];
      const double2 zj = ld2<NT>(ZB.base, (long long)j * ZB.ld + e, full);
      z.x -= h * zj.x;
      z.y -= h * zj.y;
    }
    z.x *= inv;
    z.y *= inv;
    if (!act) z = make_double2(0.0, 0.0);
    double2 u;
    if (gmf) {
      double r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int q = 0; q < kGmRaw; ++q) {
        if (q < pc.nv) {
          r0 += pc.cf[q] * (double)vq[q].x;
          r1 += pc.cf[q] * (double)vq[q].y;
        }
      }
      u = make_double2((double)dv.x * r0, (double)dv.y * r1);
    } else {
      u = make_double2(pc(e), full ? pc(e + 1) : 0.0);
    }
    double2 p = zp;
#pragma unroll 4
    for (int j = 0; j < n; ++j) {
      const double h = s_h[j];
      const long long oj = (long long)j * P.ld + e;
      const double2 pj = ld2<NT>(P.base, oj, full);
      const double2 uj = ld2<NT>(U.base, (long long)j * U.ld + e, full);
      p.x -= h * pj.x;
      p.y -= h * pj.y;
      u.x -= h * uj.x;
      u.y -= h * uj.y;
      const double d = wave_sum(pj.x * z.x + pj.y * z.y);
      if (lane == 0) s_dot[wid][j] += d;
    }
    p.x *= inv;
    p.y *= inv;
    u.x *= inv;
    u.y *= inv;
    if (!act) continue;
    st2<NT>(pn, e, p, full);
    st2<NT>(un, e, u, full);
    st2<NT>(zn, e, z, full);
    st2<NT>(zin, e, z, full);
    dp += p.x * z.x + p.y * z.y;
    zz += z.x * z.x + z.y * z.y;
  }
  {
    const double a0 = wave_sum(dp), a1 = wave_sum(zz);
    if (lane == 0) { s_dot[wid][n] = a0; s_dot[wid][n + 1] = a1; }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n + 2; c += kBlock) {
    double acc = 0.0;
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) acc += s_dot[wv][c];
    part[(long long)c * bk.n + bk.id] = acc;
  }
}
__device__ __forceinline__ void pgm_update_body(Blk bk, long long N, Window P, Window U, Window ZB, PcOutDesc pd, const double* __restrict__ wb,
             double* __restrict__ zin, double* part, SolveState* st) {
  if (st->nt) pgm_update_body_t<true>(bk, N, P, U, ZB, pd, wb, zin, part, st);
  else pgm_update_body_t<false>(bk, N, P, U, ZB, pd, wb, zin, part, st);
}
__global__ void __launch_bounds__(kBlock)
k_pgm_update(long long N, Window P, Window U, Window ZB, PcOutDesc pd, const double* __restrict__ wb,
             double* __restrict__ zin, double* part, SolveState* st) {
  pgm_update_body(this_blk(), N, P, U, ZB, pd, wb, zin, part, st);
}

// ---------------------------------------------------------------------------
// Shift estimate for PIPEFGMRES: power steps v <- A B(v) / ||A B(v)||
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_fill(long long N, double* __restrict__ v, double val) {
  for (long long e = gtid(); e < N; e += gstride()) v[e] = val;
}

// partials <v, w>, <w, w>
__global__ void __launch_bounds__(kBlock)
k_dot2(long long N, const double* __restrict__ v, const double* __restrict__ w, double* part) {
  double acc[2] = {0.0, 0.0};
  for (long long e = gtid(); e < N; e += gstride()) {
    acc[0] += v[e] * w[e];
    acc[1] += w[e] * w[e];
  }
  block_partials<2>(acc, 2, part, gridDim.x);
}

// lambda = <v, w> (v has unit norm); v = w / ||w|| (every workgroup reduces the partials).
__global__ void __launch_bounds__(kBlock)
k_power_step(long long N, const double* part, int P, double* __restrict__ v, const double* __restrict__ w,
             SolveState* st) {
  const double vw = block_sum_column(part, P, 0);
  const double ww = block_sum_column(part, P, 1);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->sigma = vw;
  if (!(ww > 0.0)) return;
  const double sc = 1.0 / sqrt(ww);
  for (long long e = gtid(); e < N; e += gstride()) v[e] = w[e] * sc;
}

}  // namespace pfk
