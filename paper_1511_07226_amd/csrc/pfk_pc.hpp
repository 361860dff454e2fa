// Preconditioner kernels B(v) for the flexible outer methods.
//
// The input is v = c1*X1 + c2*X2 (X2 may be null), formed on the fly.  The
// output is consumed by the next kernel of the outer method through a PcOut
// descriptor, so the last inner step and the outer method's use of B(v) run
// in one pass.
//
// Global k-step Jacobi-PCG (PCG of Alg. 3 with M = diag(A), from y = 0):
//   A_1 : p_1 = D^-1 v, q = A p_1;           partials <p_1,q>, <v,p_1>
//   B_j : alpha_j = gamma_j / <p_j,q>;  rho -= alpha_j q;
//         partial gamma_{j+1} = <rho, D^-1 rho>;  the last one (j = k-1)
//         also forms y = sum_{i<k} alpha_i p_i from the stored directions
//   A_j : beta_j = gamma_j/gamma_{j-1};  p_j = D^-1 rho + beta_j p_{j-1};
//         q = A p_j;  partial <p_j,q>                            (2 <= j <= k)
//   tail: y + alpha_k p_k, folded into the consumer.
// Global k-step right-Jacobi GMRES (one GMRES(k) cycle on A D^-1 t = v from
// t = 0, classical Gram-Schmidt; the basis is stored unnormalised with its
// scales in PcScalars::vs):
//   GF_j: h(., j-1) from the previous step's partials; stored V_j formed
//         (V_0 = v), w~_j = A D^-1 V_j;  partials ||V_j||^2, <V_q, w~_j>
//   GE  : the last column and the least squares on the (k+1) x k
//         Hessenberg by Givens rotations, once; the consumer forms
//         B(v) = D^-1 sum c_j V_j.
// Guards as in the definition: a zero preconditioned residual returns 0 and
// a non-positive curvature <p,q> returns the current iterate; the stop is
// recorded per step in PcScalars so later steps leave y untouched.
//
// Precision: the kernels are templated on the arithmetic type T of the inner
// sweeps and the operator description G.  FP64 uses the outer operator; the
// mixed form runs the sweeps in FP32 on BF16-stored viscosity (FP32 velocity
// and D^-1).  Conversions happen only at the boundary: v enters as FP64 and is
// rounded to T, B(v) leaves as T widened to FP64.  Reductions accumulate in
// FP64 in every form.
#pragma once
#include "pfk_state.hpp"

namespace pfk {

enum PcKind : int { kPcNone = 0, kPcJacobi = 1, kPcJacobiPcg = 2, kPcJacobiGmres = 3, kPcBlockPcg = 4 };

// Host-filled description of where B(v) comes from.
struct PcOutDesc {
  int kind;
  int k;                        // inner iterations
  int fp32;                     // inner sweeps in FP32 (float buffers below)
  const double* X1; double c1;  // v = c1*X1 + c2*X2
  const double* X2; double c2;
  const double* dinv;           // FP64 D^-1 (kinds none / jacobi)
  const void* dinv_in;          // D^-1 of the inner sweeps (T)
  const void* y;                // inner iterate (PCG), or final output (block PCG) (T)
  const void* pk;               // last inner direction (PCG) (T)
  const double* part;           // partials of the last inner kernel (PCG: <p_k,q>; A_1 also <v,p_1>)
  int P;
  const void* vbase;            // inner GMRES basis (k+1 stored vectors, ldv apart) (T)
  long long ldv;
};

template <class T>
__device__ __forceinline__ double ldw(const void* p, long long t) {
  return (double)static_cast<const T*>(p)[t];
}

// Device-side evaluator of B(v) at a node, built in the consumer's prologue.
struct PcOut {
  int kind;
  int fp32;
  const double* X1; double c1;
  const double* X2; double c2;
  const double* dinv;
  const void* dinv_in;
  const void* y;
  const void* pk;
  double alpha;
  int use_y;                    // false when k == 1 (y is still zero)
  int add_p;                    // false when the inner solve stopped before step k
  const void* vbase;            // inner GMRES: B(v) = dinv * sum cf_j V_j
  long long ldv;
  int nv;
  const double* cf;             // nv coefficients (the solve's scalars)
  __device__ __forceinline__ double v(long long t) const {
    double r = c1 * X1[t];
    if (X2 != nullptr) r += c2 * X2[t];
    return r;
  }
  __device__ __forceinline__ double w(const void* p, long long t) const {
    return fp32 ? ldw<float>(p, t) : ldw<double>(p, t);
  }
  __device__ __forceinline__ double operator()(long long t) const {
    switch (kind) {
      case kPcNone: return v(t);
      case kPcJacobi: return dinv[t] * v(t);
      case kPcBlockPcg: return w(y, t);
      case kPcJacobiGmres: {
        double r = 0.0;
        for (int q = 0; q < nv; ++q) r += cf[q] * w(vbase, (long long)q * ldv + t);
        return w(dinv_in, t) * r;
      }
      default: {
        double r = use_y ? w(y, t) : 0.0;
        if (add_p) r += alpha * w(pk, t);
        return r;
      }
    }
  }
  // The same value with the kind K and the inner storage type fixed at
  // compile time (K < 0: decided at run time); the arithmetic is that of
  // operator(), so every caller rounds alike.
  template <int K, int F32>
  __device__ __forceinline__ double at(long long t) const {
    if constexpr (K == kPcBlockPcg) {
      return F32 ? ldw<float>(y, t) : ldw<double>(y, t);
    } else if constexpr (K == kPcJacobiPcg) {
      double r = use_y ? (F32 ? ldw<float>(y, t) : ldw<double>(y, t)) : 0.0;
      if (add_p) r += alpha * (F32 ? ldw<float>(pk, t) : ldw<double>(pk, t));
      return r;
    } else {
      return (*this)(t);
    }
  }
};

// Finish the inner solve (PCG: alpha_k from the last A_k partials; GMRES:
// the small least squares) or pass through.  Every thread of the workgroup
// must call this.
__device__ __forceinline__ PcOut make_pc_out(const PcOutDesc& d, PcScalars* pcs) {
  PcOut o;
  o.kind = d.kind; o.fp32 = d.fp32;
  o.X1 = d.X1; o.c1 = d.c1; o.X2 = d.X2; o.c2 = d.c2; o.dinv = d.dinv; o.dinv_in = d.dinv_in;
  o.y = d.y; o.pk = d.pk; o.alpha = 0.0; o.use_y = d.k > 1; o.add_p = 0;
  if (d.kind == kPcJacobiPcg) {
    const double pq = block_sum_column(d.part, d.P, 0);
    double gk;
    int stopped;
    if (d.k == 1) {
      gk = block_sum_column(d.part, d.P, 1);
      stopped = (gk == 0.0);
    } else {
      gk = pcs->gamma[d.k];
      stopped = pcs->stopped[d.k - 1];
    }
    stopped = stopped || !(pq > 0.0);
    o.add_p = !stopped;
    o.alpha = stopped ? 0.0 : gk / pq;
  }
  o.vbase = d.vbase;
  o.ldv = d.ldv;
  o.nv = 0;
  o.cf = nullptr;
  if (d.kind == kPcJacobiGmres) {
    // the least squares was solved once, at the end of the inner solve; its
    // coefficients are copied to LDS (the per-node loops read them there)
    __shared__ double s_cf[kMaxInnerGmres];
    const int nv = pcs->nv;
    if (threadIdx.x < nv) s_cf[threadIdx.x] = pcs->cf[threadIdx.x];
    __syncthreads();
    o.nv = nv;
    o.cf = s_cf;
  }
  return o;
}

// B(v) + c3*X3 as a stencil input for an inner GMRES output with FP32 storage
// and at most kGmRaw basis vectors (gm_raw_ok): the basis values, D^-1 and
// X3 are loaded ahead and combined with PcOut's arithmetic when their plane
// is reached.
constexpr int kGmRaw = 8;
__device__ __forceinline__ bool gm_raw_ok(const PcOut& pc) {
  return pc.kind == kPcJacobiGmres && pc.fp32 && pc.nv <= kGmRaw;
}
struct GmRaw {
  float d;
  float v[kGmRaw];
  double x3;
};
__device__ __forceinline__ auto gm_raw_in(const PcOut& pc, const double* X3, double c3) {
  const float* V = static_cast<const float*>(pc.vbase);
  const float* D = static_cast<const float*>(pc.dinv_in);
  const int nv = pc.nv;
  const long long ldv = pc.ldv;
  const double* cf = pc.cf;
  auto load = [=](long long t) {
    GmRaw q{};
    q.d = D[t];
#pragma unroll
    for (int j = 0; j < kGmRaw; ++j)
      if (j < nv) q.v[j] = V[(long long)j * ldv + t];
    if (X3 != nullptr) q.x3 = X3[t];
    return q;
  };
  auto value = [=](const GmRaw& q) {
    double r = 0.0;
#pragma unroll
    for (int j = 0; j < kGmRaw; ++j)
      if (j < nv) r += cf[j] * (double)q.v[j];
    double v = (double)q.d * r;
    if (X3 != nullptr) v += c3 * q.x3;
    return v;
  };
  return stencil_in(load, value);
}

// ---- A_1: p_1 = D^-1 v, q = A p_1 -------------------------------------------
template <class T, class G>
__device__ __forceinline__ void pcg_a1_body(Blk bk, G g, StencilGeom sg, const T* __restrict__ dinv,
         const double* X1, double c1, const double* X2, double c2,
         T* __restrict__ pout, T* __restrict__ qout,
         double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  double acc[2] = {0.0, 0.0};
  // v at the thread's own nodes, from the plane step that loads it (keep) to
  // the one that has p_1 and q there (sink), in thread-private LDS: the dot
  // <v, p_1> reads no vector a second time
  __shared__ T s_vk[4][kBlock];
  const int tid = threadIdx.x;
  auto V = [&](double x1, double x2) { double r = c1 * x1; if (X2 != nullptr) r += c2 * x2; return T(r); };
  struct Raw { T d; double x1, x2; };
  auto load = [&](long long t) {
    Raw q{};
    q.d = dinv[t];
    q.x1 = X1[t];
    if (X2 != nullptr) q.x2 = X2[t];
    return q;
  };
  auto value = [&](const Raw& q) { return q.d * V(q.x1, q.x2); };
  auto keep = [&](long long, const Raw& q, int slot) { s_vk[slot][tid] = V(q.x1, q.x2); };
  const auto in = stencil_in(load, value, keep);
  // nontemporal stores on large systems: the halo lines that neighbouring
  // tiles still read stay longer in the L2 (256^3, one geometry: FETCH of
  // A_j 1.23 -> 1.19x its algorithmic reads, of A_1 1.38 -> 1.32x)
  const bool nt = st->nt != 0;
  auto sink = [&](long long idx, T pc, T q, int slot) {
    if (nt) {
      stnt(pout + idx, pc);
      stnt(qout + idx, q);
    } else {
      pout[idx] = pc;
      qout[idx] = q;
    }
    acc[0] += (double)pc * (double)q;
    acc[1] += (double)s_vk[slot][tid] * (double)pc;
  };
  // FP32 loads two plane steps ahead (no occupancy step lost; mixed PIPEFCG
  // 213 -> 227 it/s at 256^3); FP64 one (a second plane would cost one)
  stencil_march<T, 0, sizeof(T) == 4 ? 2 : 1>(g, sg, bk.id, in, sink);
  block_partials<2>(acc, 2, part, bk.n, bk.id);
}
template <class T, class G>
__global__ void __launch_bounds__(kBlock)
k_pcg_a1(G g, StencilGeom sg, const T* __restrict__ dinv,
         const double* X1, double c1, const double* X2, double c2,
         T* __restrict__ pout, T* __restrict__ qout,
         double* part, const SolveState* st) {
  pcg_a1_body(this_blk(), g, sg, dinv, X1, c1, X2, c2, pout, qout, part, st);
}

// ---- B_j (1 <= j < k): rho -= alpha q, partial <rho, D^-1 rho> ---------------
// The iterate y = sum_{i<k} alpha_i p_i is formed once, by the last B
// (j = k-1), from the stored directions p_1 .. p_{k-1} (slot i-1 of P) and
// the step lengths the earlier B's recorded: the accumulation
// y += alpha_i p_i in the same order and type as a running update, without
// reading and writing y at every step (k = 5 at 256^3: six fewer vector
// passes per inner solve).  A stopped step (zero or non-positive curvature)
// leaves rho and y as they are, as does every later one.
template <class T>
__device__ __forceinline__ void pcg_b_body(Blk bk, int jstep, int k, long long N, const T* __restrict__ dinv,
        const double* X1, double c1, const double* X2, double c2,
        const T* Pbase, long long ldp, const T* __restrict__ q,
        T* __restrict__ rho, T* __restrict__ y,
        const double* part_in, int P_in, double* part_out, SolveState* st) {
  if (!wg_running(st)) return;
  PcScalars* pcs = &st->pc;
  const double pq = block_sum_column(part_in, P_in, 0);
  double gj;
  int stopped;
  if (jstep == 1) {
    gj = block_sum_column(part_in, P_in, 1);
    stopped = (gj == 0.0);
  } else {
    gj = pcs->gamma[jstep];
    stopped = pcs->stopped[jstep - 1];
  }
  stopped = stopped || !(pq > 0.0);
  const T alpha = T(stopped ? 0.0 : gj / pq);
  if (bk.id == 0 && threadIdx.x == 0) {
    if (jstep == 1) pcs->gamma[1] = gj;
    pcs->stopped[jstep] = stopped;
    pcs->alpha[jstep] = (double)alpha;
  }
  const bool last = jstep + 1 == k;
  // the earlier steps' lengths (their stops are monotone: once stopped, every
  // later step is); those with a stop contribute nothing
  __shared__ double s_al[kMaxInner + 2];
  __shared__ int s_nl;    // leading steps that contribute to y
  if (last) {
    if (threadIdx.x == 0) {
      int nl = 0;
      for (int i = 1; i < jstep; ++i) {
        if (pcs->stopped[i]) break;
        s_al[i] = pcs->alpha[i];
        nl = i;
      }
      if (nl == jstep - 1 && !stopped) {
        s_al[jstep] = (double)alpha;
        nl = jstep;
      }
      s_nl = nl;
    }
    __syncthreads();
  }
  const int nl = last ? s_nl : 0;
  double acc[1] = {0.0};
  // VW nodes per lane (16-byte accesses to the T vectors; all vectors start
  // 16-byte aligned), the scalar tail after; nontemporal accesses for vectors
  // far larger than the caches (st->nt).  The arithmetic per node is the same.
  constexpr int VW = 16 / sizeof(T);
  typedef T tv_t __attribute__((ext_vector_type(VW)));
  typedef double dv_t __attribute__((ext_vector_type(VW), aligned(16)));   // X1, X2 16-byte aligned
  auto sweep = [&](auto ntc) {
    constexpr bool NT = decltype(ntc)::value;
    auto ld = [](const auto* a) {
      if constexpr (NT) return ldnt(a);
      else return *a;
    };
    auto sto = [](auto* a, auto v) {
      if constexpr (NT) stnt(a, v);
      else *a = v;
    };
    const long long nv = N / VW;
    for (long long qv = bk.gtid(); qv < nv; qv += bk.gstride()) {
      const long long e = qv * VW;
      tv_t r;
      if (jstep == 1) {
        const dv_t x1 = ld(reinterpret_cast<const dv_t*>(X1 + e));
        dv_t x2 = {};
        if (X2 != nullptr) x2 = ld(reinterpret_cast<const dv_t*>(X2 + e));
#pragma unroll
        for (int l = 0; l < VW; ++l) {
          double rv = c1 * x1[l];
          if (X2 != nullptr) rv += c2 * x2[l];
          r[l] = T(rv);
        }
      } else {
        r = ld(reinterpret_cast<const tv_t*>(rho + e));
      }
      tv_t qv4 = {};
      if (!stopped) qv4 = ld(reinterpret_cast<const tv_t*>(q + e));
      const tv_t dv = ld(reinterpret_cast<const tv_t*>(dinv + e));
      tv_t ro;
#pragma unroll
      for (int l = 0; l < VW; ++l) {
        T rl = r[l];
        if (!stopped) rl -= alpha * qv4[l];
        ro[l] = rl;
        acc[0] += (double)rl * (double)(dv[l] * rl);
      }
      sto(reinterpret_cast<tv_t*>(rho + e), ro);
      if (last) {
        tv_t yv = {};
#pragma unroll 4
        for (int i = 1; i <= nl; ++i) {
          const T ai = T(s_al[i]);
          const tv_t pi = ld(reinterpret_cast<const tv_t*>(Pbase + (long long)(i - 1) * ldp + e));
#pragma unroll
          for (int l = 0; l < VW; ++l) yv[l] += ai * pi[l];
        }
        sto(reinterpret_cast<tv_t*>(y + e), yv);
      }
    }
    for (long long e = nv * VW + bk.gtid(); e < N; e += bk.gstride()) {
      T r;
      if (jstep == 1) {
        double rv = c1 * ld(X1 + e);
        if (X2 != nullptr) rv += c2 * ld(X2 + e);
        r = T(rv);
      } else {
        r = ld(rho + e);
      }
      if (!stopped) r -= alpha * ld(q + e);
      const T dv = ld(dinv + e);
      acc[0] += (double)r * (double)(dv * r);
      sto(rho + e, r);
      if (last) {
        T yv = T(0);
        for (int i = 1; i <= nl; ++i) yv += T(s_al[i]) * ld(Pbase + (long long)(i - 1) * ldp + e);
        sto(y + e, yv);
      }
    }
  };
  if (st->nt) sweep(std::true_type{});
  else sweep(std::false_type{});
  block_partials<1>(acc, 1, part_out, bk.n, bk.id);
}
template <class T>
__global__ void __launch_bounds__(kBlock)
k_pcg_b(int jstep, int k, long long N, const T* __restrict__ dinv,
        const double* X1, double c1, const double* X2, double c2,
        const T* Pbase, long long ldp, const T* __restrict__ q,
        T* __restrict__ rho, T* __restrict__ y,
        const double* part_in, int P_in, double* part_out, SolveState* st) {
  pcg_b_body(this_blk(), jstep, k, N, dinv, X1, c1, X2, c2, Pbase, ldp, q, rho, y, part_in, P_in, part_out, st);
}

// ---- A_j (2 <= j <= k): p_j = D^-1 rho + beta p_{j-1}, q = A p_j -------------
template <class T, class G>
__device__ __forceinline__ void pcg_a_body(Blk bk, int jstep, G g, StencilGeom sg, const T* __restrict__ dinv,
        const T* __restrict__ rho, const T* __restrict__ pprev,
        T* __restrict__ pout, T* __restrict__ qout,
        const double* part_in, int P_in, double* part_out, SolveState* st) {
  if (!wg_running(st)) return;
  PcScalars* pcs = &st->pc;
  const double gj = block_sum_column(part_in, P_in, 0);
  const double gprev = pcs->gamma[jstep - 1];
  const int stopped = pcs->stopped[jstep - 1];
  const T beta = T((stopped || gprev == 0.0) ? 0.0 : gj / gprev);
  if (bk.id == 0 && threadIdx.x == 0) pcs->gamma[jstep] = gj;
  double acc[1] = {0.0};
  struct Raw { T d, r, p; };
  const auto in = stencil_in([&](long long t) { return Raw{dinv[t], rho[t], pprev[t]}; },
                             [&](const Raw& q) { return q.d * q.r + beta * q.p; });
  // nontemporal stores on large systems: the halo lines that neighbouring
  // tiles still read stay longer in the L2 (256^3, one geometry: FETCH of
  // A_j 1.23 -> 1.19x its algorithmic reads, of A_1 1.38 -> 1.32x)
  const bool nt = st->nt != 0;
  auto sink = [&](long long idx, T pc, T q) {
    if (nt) {
      stnt(pout + idx, pc);
      stnt(qout + idx, q);
    } else {
      pout[idx] = pc;
      qout[idx] = q;
    }
    acc[0] += (double)pc * (double)q;
  };
  // FP32 loads two plane steps ahead (no occupancy step lost; mixed PIPEFCG
  // 213 -> 227 it/s at 256^3); FP64 one (a second plane would cost one)
  stencil_march<T, 0, sizeof(T) == 4 ? 2 : 1>(g, sg, bk.id, in, sink);
  block_partials<1>(acc, 1, part_out, bk.n, bk.id);
}
template <class T, class G>
__global__ void __launch_bounds__(kBlock)
k_pcg_a(int jstep, G g, StencilGeom sg, const T* __restrict__ dinv,
        const T* __restrict__ rho, const T* __restrict__ pprev,
        T* __restrict__ pout, T* __restrict__ qout,
        const double* part_in, int P_in, double* part_out, SolveState* st) {
  pcg_a_body(this_blk(), jstep, g, sg, dinv, rho, pprev, pout, qout, part_in, P_in, part_out, st);
}

// ---- inner GMRES -----------------------------------------------------------
// Right-Jacobi GMRES(k) from x = 0 (Arnoldi with classical Gram-Schmidt).
// The basis is stored unnormalised: stored vector q is nu_q V_q with
// nu_q = ||stored q|| (vs[q] = 1/nu_q), and the operator is applied to the
// stored vector, w~_j = A D^-1 (stored j) = nu_j A D^-1 V_j.  One stencil
// pass GF_j per step j: the stored vector j is formed at every node from the
// previous step's data -- j = 0: v = c1 X1 + c2 X2; j >= 1:
// vs[j-1] w~_{j-1} - sum_{q<j} h(q,j-1) vs[q] (stored q), which is
// w_{j-1} - sum h(q,j-1) V_q -- stored, its squared norm summed, and
// w~_j = A D^-1 (stored j) computed from it; where w~_j of a node is known,
// the node's stored vectors 0..j (read or formed two plane steps earlier and
// held in thread-private LDS since) give its terms of <stored q, w~_j>.
// GF_j's partials: column 0 ||stored j||^2, column 1 + q <stored q, w~_j>
// (q <= j), and at the last step column j + 2 ||w~_j||^2.  GF_{j+1} takes
// nu_j from column 0 (beta0 for j = 0, else the subdiagonal h(j,j-1)) and
// h(q,j) = vs[q] vs[j] <stored q, w~_j> from the others.
// GE (one workgroup) finishes: nu_{k-1}, column k-1, its subdiagonal
// h(k,k-1) and the least squares, whose coefficients the consumers read.  A
// zero norm nu_j ends the cycle at j columns (beta0 = 0 gives B(v) = 0, a
// zero subdiagonal is a happy breakdown).  w~ alternates between two
// buffers (GF_j reads one at halo nodes while writing the other), and so do
// the partials.

// Column `col` of the Hessenberg from GF_col's partials: nu_col (into the
// scalars: beta0 or h(col,col-1), vs[col]; a zero norm ends the cycle at col
// columns and returns false), h(q,col) into the scalars, and the
// coefficients of the next stored vector, cw = vs[col] for w~_col and
// c[q] = h(q,col) vs[q].  Workgroup 0 writes the scalars; every workgroup
// sums the same partials in the same order, so all take the same values.
// Every thread calls it.
__device__ __forceinline__ bool gm_column(Blk bk, int col, const double* part, int P, PcScalars* pcs,
                                          double* c, double& cw) {
  __shared__ double s_col[kMaxInnerGmres + 1];
  block_sum_columns(part, P, col + 2, s_col);
  const double nrm = sqrt(s_col[0]);
  const double sc = nrm == 0.0 ? 0.0 : 1.0 / nrm;
  if (bk.id == 0 && threadIdx.x == 0) {
    if (col == 0) pcs->beta0 = nrm;
    else pcs->h[(col - 1) * (kMaxInner + 1) + col] = nrm;
    pcs->vs[col] = sc;
    if (nrm == 0.0) pcs->ncol = col;
  }
  if (nrm == 0.0) return false;
  if (threadIdx.x == 0) {
    for (int q = 0; q <= col; ++q) {
      const double vq = q == col ? sc : pcs->vs[q];
      const double hq = vq * sc * s_col[1 + q];
      c[q] = hq * vq;
      if (bk.id == 0) pcs->h[col * (kMaxInner + 1) + q] = hq;
    }
  }
  __syncthreads();
  cw = sc;
  return true;
}

// Raw loads of GF_J at a node: D^-1 and, for J >= 1, w~_{J-1} and the first
// RJ stored vectors (RJ = J for J <= kGfFixed, else kMaxInnerGmres - 1 with
// the count taken at run time); for J = 0 the outer input v.
constexpr int kGfFixed = 4;
template <class T, int J>
struct GfRaw {
  static constexpr int RJ = J <= kGfFixed ? J : kMaxInnerGmres - 1;
  T d, w;
  T v[RJ > 0 ? RJ : 1];
};
template <class T>
struct GfRaw<T, 0> {
  static constexpr int RJ = 0;
  T d;
  double x1, x2;
};

// WW: the last step of the cycle, which also sums ||w~_j||^2.
template <class T, class G, int CV, int J, bool WW>
__device__ __forceinline__ void gmpc_fused_body(Blk bk, int jstep, int k, G g, StencilGeom sg,
                                                const T* __restrict__ dinv, const double* X1, double c1,
                                                const double* X2, double c2, T* Vbase, long long ldv,
                                                const T* wprev, T* __restrict__ wout, const double* part_in,
                                                int P_in, double* part_out, SolveState* st) {
  if (!wg_running(st)) return;
  PcScalars* pcs = &st->pc;
  using R = GfRaw<T, J>;
  constexpr int RJ = R::RJ;
  // columns: 0 ||stored j||^2, 1 + q <stored q, w~_j> for q < RJ, 1 + RJ
  // <stored j, w~_j>, with WW 2 + RJ ||w~_j||^2 (moved to 1 + j and 2 + j at
  // the end when the basis length is taken at run time)
  constexpr int NC = RJ + (WW ? 3 : 2);
  double acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = 0.0;
  // the squared norms (columns 0 and 2 + RJ) accumulate in thread-private
  // LDS: two fewer live registers keep these kernels at four workgroups per
  // CU (the same additions in the same order as in a register)
  __shared__ double s_nn[WW ? 2 : 1][kBlock];
  // the thread's stored vectors 0..j of its nodes, from keep to sink: four
  // node slots (plane parity, row), one entry per thread, so no barrier
  __shared__ T s_v[4][RJ + 1][kBlock];
  const int tid = threadIdx.x;
  s_nn[0][tid] = 0.0;
  if constexpr (WW) s_nn[WW][tid] = 0.0;
  T* Vj = Vbase + (long long)jstep * ldv;
  auto sink = [&](long long idx, T, T Au, int slot) {
    wout[idx] = Au;
    const double wa = (double)Au;
#pragma unroll
    for (int p = 0; p < RJ; ++p)
      if (J <= kGfFixed || p < jstep) acc[1 + p] += (double)s_v[slot][p][tid] * wa;
    acc[1 + RJ] += (double)s_v[slot][RJ][tid] * wa;
    if constexpr (WW) s_nn[WW][tid] = s_nn[WW][tid] + wa * wa;
  };
  // FP32 with up to two basis terms: loads two plane steps ahead; longer
  // bases take one step (the second plane of raw loads would cost an
  // occupancy step: at 256^3, J = 3 and 4 ran 1-4% faster with one)
  constexpr int PD = (sizeof(T) == 4 && J <= 2) ? 2 : 1;
  if constexpr (J == 0) {
    if (bk.id == 0 && threadIdx.x == 0) pcs->ncol = k;
    auto load = [&](long long t) {
      R q;
      q.d = dinv[t];
      q.x1 = X1[t];
      q.x2 = X2 != nullptr ? X2[t] : 0.0;
      return q;
    };
    auto form = [&](const R& q) {
      double v = c1 * q.x1;
      if (X2 != nullptr) v += c2 * q.x2;
      return T(v);
    };
    auto value = [&](const R& q) { return q.d * form(q); };
    auto keep = [&](long long t, const R& q, int slot) {
      const T v = form(q);
      Vj[t] = v;
      s_v[slot][0][tid] = v;
      s_nn[0][tid] = s_nn[0][tid] + (double)v * (double)v;
    };
    stencil_march<T, CV, PD>(g, sg, bk.id, stencil_in(load, value, keep), sink);
  } else {
    // an earlier step ended the cycle (workgroup 0 of this launch may be
    // writing ncol: gm_column below ends it at jstep - 1 columns)
    if (jstep >= wg_load(&pcs->ncol)) return;
    __shared__ double s_c[kMaxInnerGmres];
    double cwd;
    if (!gm_column(bk, jstep - 1, part_in, P_in, pcs, s_c, cwd)) return;
    const T cw = T(cwd);
    T c[RJ];
#pragma unroll
    for (int q = 0; q < RJ; ++q) c[q] = q < jstep ? T(s_c[q]) : T(0);
    auto load = [&](long long t) {
      R q;
      q.d = dinv[t];
      q.w = wprev[t];
#pragma unroll
      for (int p = 0; p < RJ; ++p) q.v[p] = (J <= kGfFixed || p < jstep) ? Vbase[(long long)p * ldv + t] : T(0);
      return q;
    };
    auto form = [&](const R& q) {
      T v = cw * q.w;
#pragma unroll
      for (int p = 0; p < RJ; ++p)
        if (J <= kGfFixed || p < jstep) v -= c[p] * q.v[p];
      return v;
    };
    auto value = [&](const R& q) { return q.d * form(q); };
    auto keep = [&](long long t, const R& q, int slot) {
      const T v = form(q);
      Vj[t] = v;
#pragma unroll
      for (int p = 0; p < RJ; ++p)
        if (J <= kGfFixed || p < jstep) s_v[slot][p][tid] = q.v[p];
      s_v[slot][RJ][tid] = v;
      s_nn[0][tid] = s_nn[0][tid] + (double)v * (double)v;
    };
    stencil_march<T, CV, PD>(g, sg, bk.id, stencil_in(load, value, keep), sink);
  }
  acc[0] = s_nn[0][tid];
  if constexpr (WW) acc[NC - 1] = s_nn[WW][tid];
  if constexpr (J > kGfFixed) {
    // basis length at run time: <stored j, w~_j> and ||w~_j||^2 to columns
    // 1 + j and 2 + j (the columns between are zero)
    const double dj = acc[1 + RJ], ww = WW ? acc[NC - 1] : 0.0;
    acc[1 + RJ] = 0.0;
    if constexpr (WW) acc[NC - 1] = 0.0;
#pragma unroll
    for (int q = 1 + kGfFixed; q < NC; ++q) {
      if (q == 1 + jstep) acc[q] = dj;
      if (WW && q == 2 + jstep) acc[q] = ww;
    }
  }
  block_partials<NC>(acc, jstep + (WW ? 3 : 2), part_out, bk.n, bk.id);
}
template <class T, class G, int CV, int J, bool WW>
__global__ void __launch_bounds__(kBlock)
k_gmpc_fused(int jstep, int k, G g, StencilGeom sg, const T* __restrict__ dinv, const double* X1, double c1,
             const double* X2, double c2, T* Vbase, long long ldv, const T* wprev, T* __restrict__ wout,
             const double* part_in, int P_in, double* part_out, SolveState* st) {
  gmpc_fused_body<T, G, CV, J, WW>(this_blk(), jstep, k, g, sg, dinv, X1, c1, X2, c2, Vbase, ldv, wprev, wout,
                                   part_in, P_in, part_out, st);
}

// GE: the end of the inner solve, one workgroup.  From GF_{k-1}'s partials:
// nu_{k-1} (a zero norm ends the cycle at k-1 columns), column k-1 of the
// Hessenberg, and its subdiagonal from the Pythagorean identity
// h(k,k-1)^2 = ||w_{k-1}||^2 - sum_q h(q,k-1)^2 (exact for an orthonormal
// basis, as PIPEFGMRES takes its own norms; a value <= 0 counts as a happy
// breakdown, h = 0); then the small least squares min || beta0 e_0 - H y ||
// over the active columns (Givens rotations), stored as cf[q] = y_q vs[q]
// for the consumers.
__device__ __forceinline__ void gmpc_finish_body(int k, const double* part, int P, SolveState* st) {
  if (!wg_running(st)) return;
  PcScalars* pcs = &st->pc;
  constexpr int L = kMaxInner + 1, M = kMaxInnerGmres + 1;
  __shared__ double s_col[kMaxInnerGmres + 2];
  __shared__ double H[M * kMaxInnerGmres];
  __shared__ double g[M], cs[kMaxInnerGmres], sn[kMaxInnerGmres], yv[kMaxInnerGmres];
  // ||stored k-1||^2, <stored q, w~_{k-1}> for q < k, ||w~_{k-1}||^2
  if (pcs->ncol == k) block_sum_columns(part, P, k + 2, s_col);
  if (threadIdx.x != 0) return;
  int nc = pcs->ncol;
  double hk = 0.0;
  if (nc == k) {
    const double nrm = sqrt(s_col[0]);
    const double sc = nrm == 0.0 ? 0.0 : 1.0 / nrm;
    if (k == 1) pcs->beta0 = nrm;
    else pcs->h[(k - 2) * L + k - 1] = nrm;
    pcs->vs[k - 1] = sc;
    if (nrm == 0.0) {
      nc = k - 1;
      pcs->ncol = nc;
    } else {
      double t = sc * sc * s_col[k + 1];
      for (int q = 0; q < k; ++q) {
        const double vq = q == k - 1 ? sc : pcs->vs[q];
        const double hq = vq * sc * s_col[1 + q];
        pcs->h[(k - 1) * L + q] = hq;
        t -= hq * hq;
      }
      hk = t > 0.0 ? sqrt(t) : 0.0;
    }
  }
  for (int jj = 0; jj < nc; ++jj)
    for (int ii = 0; ii <= jj + 1; ++ii) H[jj * M + ii] = pcs->h[jj * L + ii];
  if (nc == k && nc > 0) H[(nc - 1) * M + nc] = hk;
  for (int ii = 0; ii <= nc; ++ii) g[ii] = 0.0;
  g[0] = pcs->beta0;
  for (int jj = 0; jj < nc; ++jj) {
    double* col = &H[jj * M];
    for (int ii = 0; ii < jj; ++ii) {
      const double a = col[ii], b = col[ii + 1];
      col[ii] = cs[ii] * a + sn[ii] * b;
      col[ii + 1] = -sn[ii] * a + cs[ii] * b;
    }
    const double a = col[jj], b = col[jj + 1];
    const double dd = hypot(a, b);
    cs[jj] = dd == 0.0 ? 1.0 : a / dd;
    sn[jj] = dd == 0.0 ? 0.0 : b / dd;
    col[jj] = dd;
    col[jj + 1] = 0.0;
    const double gi = g[jj];
    g[jj] = cs[jj] * gi;
    g[jj + 1] = -sn[jj] * gi;
  }
  for (int ii = nc - 1; ii >= 0; --ii) {
    double acc = g[ii];
    for (int jj = ii + 1; jj < nc; ++jj) acc -= H[jj * M + ii] * yv[jj];
    yv[ii] = acc / H[ii * M + ii];
  }
  for (int ii = 0; ii < nc; ++ii) pcs->cf[ii] = yv[ii] * pcs->vs[ii];
  pcs->nv = nc;
}
__global__ void __launch_bounds__(kBlock)
k_gmpc_finish(int k, const double* part, int P, SolveState* st) {
  gmpc_finish_body(k, part, P, st);
}

// ---- block-Jacobi PCG ------------------------------------------------------
// The per-block inner solve of the experiments (section 6.2): the domain is
// cut into cubes of kBjEdge nodes per axis (squares in 2D) starting at
// interior index 0, the last block per axis ragged.  Each block runs k steps
// of Jacobi-PCG from y = 0 on its principal submatrix A_bb (couplings to
// other blocks dropped, the diagonal of A kept whole) with its own scalars
// and guards, so the whole inner solve is one kernel with no device-wide
// synchronisation: v is read once and B(v) written once.
//
// Shape: a 64-lane wave holds one 8 x 8 (x, y) plane of a block (lane =
// 8 y + x).  3D: a block is two waves of four planes each and a workgroup
// takes two x-adjacent blocks, so every 128-byte row segment of a vector is
// read by one compute unit.  2D: a wave is a whole block, four x-adjacent
// blocks per workgroup.  The block's coefficients (diagonal, D^-1 and the six
// in-block off-diagonals) are formed once from the viscosity and velocities
// and stay in registers; directions are exchanged through LDS.  Block dot
// products accumulate in FP64: a DPP sum over the wave read back from its
// last lane (every lane takes the same value) and, in 3D, the block's two
// wave sums through LDS in a fixed order.
constexpr int kBjEdge = 8;

template <int D3>
struct BjShape {
  static constexpr int NPT = D3 ? 4 : 1;        // planes (nodes) per thread
  static constexpr int WPB = D3 ? 2 : 1;        // waves per block
  static constexpr int BPW = kWaves / WPB;      // blocks per workgroup (along x)
  static constexpr int ZL = D3 ? kBjEdge : 1;   // planes per block
};

// Diagonal and in-block off-diagonal couplings of node (i, j, k); zl is its
// plane within the block.  (A_bb u)_c = d u_c - sum_f o_f u_f, faces in the
// order x+, x-, y+, y-, z+, z-; o_f = 0 for a neighbour outside the block or
// on the boundary.
// The global loads of one node's block coefficients (viscosity at the node
// and its six neighbours; face velocities when the operator has them) and of
// its input X1, X2: loads only, so every plane's loads are in flight at once.
template <class EC, class VC>
struct BjRaw {
  EC e[7];
  VC v[6];
  double x1, x2;
};
template <class G, class EC, class VC>
__device__ __forceinline__ void bj_load(const G& g, int i, int j, int k, const double* X1, const double* X2,
                                        BjRaw<EC, VC>& r) {
  const long long pc = padded_index(g, i, j, k);
  const bool d3 = g.dim == 3;
  r.e[0] = g.eta[pc];
  r.e[1] = g.eta[pc + 1];
  r.e[2] = g.eta[pc - 1];
  r.e[3] = g.eta[pc + g.sy];
  r.e[4] = g.eta[pc - g.sy];
  if (d3) {
    r.e[5] = g.eta[pc + g.sz];
    r.e[6] = g.eta[pc - g.sz];
  }
  if (g.vel != nullptr) {
    const auto* vx = g.vel;
    const auto* vy = g.vel + g.vstride;
    const auto* vz = g.vel + 2 * g.vstride;
    r.v[0] = vx[pc];
    r.v[1] = vx[pc - 1];
    r.v[2] = vy[pc];
    r.v[3] = vy[pc - g.sy];
    if (d3) {
      r.v[4] = vz[pc];
      r.v[5] = vz[pc - g.sz];
    }
  }
  const long long e = vec_index(g, i, j, k);
  r.x1 = X1[e];
  if (X2 != nullptr) r.x2 = X2[e];
}

// A node's row of its block's matrix A_bb from the loaded values: diagonal d
// (of A, kept whole) and the in-block off-diagonal magnitudes o (x+, x-, y+,
// y-, z+, z-; zero where the neighbour is outside the block or the domain).
template <class T, class G, class EC, class VC>
__device__ __forceinline__ void bj_coeffs(const G& g, const BjRaw<EC, VC>& r, int i, int j, int k, int lx, int ly,
                                          int zl, T& d, T (&o)[6]) {
  const bool d3 = g.dim == 3;
  const T ec = T(to_real(r.e[0]));
  T kf[6];
  kf[0] = harmonic(ec, T(to_real(r.e[1])));
  kf[1] = harmonic(ec, T(to_real(r.e[2])));
  kf[2] = harmonic(ec, T(to_real(r.e[3])));
  kf[3] = harmonic(ec, T(to_real(r.e[4])));
  kf[4] = d3 ? harmonic(ec, T(to_real(r.e[5]))) : T(0);
  kf[5] = d3 ? harmonic(ec, T(to_real(r.e[6]))) : T(0);
  const bool in[6] = {lx + 1 < kBjEdge && i + 1 < g.nx, lx > 0,
                      ly + 1 < kBjEdge && j + 1 < g.ny, ly > 0,
                      d3 && zl + 1 < kBjEdge && k + 1 < g.nz, d3 && zl > 0};
  const T h2 = T(g.h2inv);
  T dd = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) dd += kf[f];
  dd *= h2;
  T vn[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  if (g.vel != nullptr) {
    vn[0] = T(to_real(r.v[0]));
    vn[1] = -T(to_real(r.v[1]));
    vn[2] = T(to_real(r.v[2]));
    vn[3] = -T(to_real(r.v[3]));
    if (d3) {
      vn[4] = T(to_real(r.v[4]));
      vn[5] = -T(to_real(r.v[5]));
    }
    T up = T(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) up += fmax(vn[f], T(0));
    dd += T(g.hinv) * up;
  }
#pragma unroll
  for (int f = 0; f < 6; ++f) o[f] = in[f] ? h2 * kf[f] - T(g.hinv) * fmin(vn[f], T(0)) : T(0);
  d = dd;
}

// B(v) for every block, v = c1*X1 + c2*X2 (FP64, rounded to T), written to
// yout (T).  Workgroups: wx * wy * wz, with wx = ceil(nx / (BPW * 8)),
// wy = ceil(ny / 8), wz = ceil(nz / 8) (1 in 2D).
template <class T, class G, int D3>
__device__ __forceinline__ void block_pcg_body(Blk bk, G g, int wx, int wy, int k, const double* X1, double c1, const double* X2, double c2,
            T* __restrict__ yout, const SolveState* st) {
  using Sh = BjShape<D3>;
  constexpr int NPT = Sh::NPT, WPB = Sh::WPB, BPW = Sh::BPW, ZL = Sh::ZL;
  if (!wg_running(st)) return;
  __shared__ T sp[BPW * ZL * 64];
  __shared__ double sred[2][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 7, ly = lane >> 3;
  const int blk = wave / WPB, zh = wave % WPB;
  const int b = bk.id;
  const int gx = b % wx, gy = (b / wx) % wy, gz = b / (wx * wy);
  const int i = (gx * BPW + blk) * kBjEdge + lx;
  const int j = gy * kBjEdge + ly;
  const bool col = i < g.nx && j < g.ny;

  T dg[NPT], dinv[NPT], o[NPT][6], r[NPT], p[NPT], q[NPT], y[NPT];
  int slot[NPT];
  bool valid[NPT];
  double acc = 0.0;
  // every plane's loads first, then the arithmetic on them
  using EC = typename std::remove_cv<typename std::remove_pointer<decltype(g.eta)>::type>::type;
  using VC = typename std::remove_cv<typename std::remove_pointer<decltype(g.vel)>::type>::type;
  BjRaw<EC, VC> raw[NPT];
#pragma unroll
  for (int n = 0; n < NPT; ++n) {
    const int zl = zh * NPT + n;
    const int kz = gz * ZL + zl;
    slot[n] = ((blk * ZL + zl) * kBjEdge + ly) * kBjEdge + lx;
    valid[n] = col && kz < g.nz;
    if (valid[n]) bj_load(g, i, j, kz, X1, X2, raw[n]);
  }
#pragma unroll
  for (int n = 0; n < NPT; ++n) {
    const int zl = zh * NPT + n;
    const int kz = gz * ZL + zl;
    y[n] = T(0);
    if (valid[n]) {
      bj_coeffs<T>(g, raw[n], i, j, kz, lx, ly, zl, dg[n], o[n]);
      dinv[n] = T(1) / dg[n];
      double v = c1 * raw[n].x1;
      if (X2 != nullptr) v += c2 * raw[n].x2;
      r[n] = T(v);
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) o[n][f] = T(0);
      dg[n] = T(1);
      dinv[n] = T(0);
      r[n] = T(0);
    }
    p[n] = dinv[n] * r[n];
    acc += (double)r[n] * (double)p[n];
  }

  int par = 0;
  auto bsum = [&](double part) -> double {
    double s = wave_sum(part);
    if (WPB == 1) return s;
    if (lane == 0) sred[par][wave] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < WPB; ++w) t += sred[par][blk * WPB + w];
    par ^= 1;
    return t;
  };

  double gamma = bsum(acc);
  bool live = gamma != 0.0;
  for (int step = 1; step <= k; ++step) {
#pragma unroll
    for (int n = 0; n < NPT; ++n) sp[slot[n]] = p[n];
    __syncthreads();
    acc = 0.0;
#pragma unroll
    for (int n = 0; n < NPT; ++n) {
      const int zl = zh * NPT + n;
      const int s = slot[n];
      const T nb0 = lx + 1 < kBjEdge ? sp[s + 1] : T(0);
      const T nb1 = lx > 0 ? sp[s - 1] : T(0);
      const T nb2 = ly + 1 < kBjEdge ? sp[s + kBjEdge] : T(0);
      const T nb3 = ly > 0 ? sp[s - kBjEdge] : T(0);
      T a = dg[n] * p[n] - (o[n][0] * nb0 + o[n][1] * nb1 + o[n][2] * nb2 + o[n][3] * nb3);
      if (D3) {
        const T nb4 = zl + 1 < kBjEdge ? sp[s + 64] : T(0);
        const T nb5 = zl > 0 ? sp[s - 64] : T(0);
        a -= o[n][4] * nb4 + o[n][5] * nb5;
      }
      q[n] = a;
      acc += (double)p[n] * (double)a;
    }
    const double pq = bsum(acc);
    live = live && pq > 0.0;
    const double alpha = live ? gamma / pq : 0.0;
    const T at = T(alpha);
#pragma unroll
    for (int n = 0; n < NPT; ++n) y[n] += at * p[n];
    if (step < k) {
      acc = 0.0;
      T z[NPT];
#pragma unroll
      for (int n = 0; n < NPT; ++n) {
        r[n] -= at * q[n];
        z[n] = dinv[n] * r[n];
        acc += (double)r[n] * (double)z[n];
      }
      const double gnew = bsum(acc);
      const T beta = T(live ? gnew / gamma : 0.0);
#pragma unroll
      for (int n = 0; n < NPT; ++n) p[n] = z[n] + beta * p[n];
      gamma = gnew;
    }
  }
#pragma unroll
  for (int n = 0; n < NPT; ++n)
    if (valid[n]) yout[vec_index(g, i, j, gz * ZL + zh * NPT + n)] = y[n];
}
template <class T, class G, int D3>
__global__ void __launch_bounds__(kBlock)
k_block_pcg(G g, int wx, int wy, int k, const double* X1, double c1, const double* X2, double c2,
            T* __restrict__ yout, const SolveState* st) {
  block_pcg_body<T, G, D3>(this_blk(), g, wx, wy, k, X1, c1, X2, c2, yout, st);
}

}  // namespace pfk
