// The seeded noisy preconditioner of the stagnation study (section 2.2.1,
// Figure 1): B(v) = v + eta ||v|| g / ||g|| with g standard normal.
//
// g is a counter-based stream, so any node's value can be computed where it
// is needed and a solve is reproducible draw for draw:
//   * Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): counter
//     (e, d, 0, 0) for node e of draw d, key (seed, 0).  A round multiplies
//     counter words 0 and 2 by two odd 64-bit constants (both 64-bit halves of
//     each product are kept), xors the high halves with words 1, 3 and the
//     key, and permutes; the key advances by two Weyl increments between the
//     ten rounds.
//   * Box-Muller on the top 53 bits of output words 0 and 1:
//     u1 = (a + 1) 2^-53 in (0, 1], u2 = b 2^-53 in [0, 1),
//     g = sqrt(-2 ln u1) cos(2 pi u2)  (one normal per counter).
//
// One application is two launches: the partial sums of ||v||^2 and ||g||^2,
// and the output y = v + s g with s = eta ||v|| / ||g|| (0 when either norm
// is 0), stored in the inner-solve output vector so consumers read it like
// block PCG's output.  A solve counts its applications on the device
// (k_noise_advance at the end of each phase).
#pragma once
#include "pfk_device.hpp"
#include "pfk_state.hpp"

namespace pfk {

__device__ __forceinline__ double noise_normal(unsigned long long seed, unsigned long long draw,
                                               unsigned long long e) {
  constexpr unsigned long long kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr unsigned long long kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  unsigned long long x0 = e, x1 = draw, x2 = 0, x3 = 0;
  unsigned long long k0 = seed, k1 = 0;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const unsigned long long h0 = __umul64hi(kM0, x0), l0 = kM0 * x0;
    const unsigned long long h2 = __umul64hi(kM1, x2), l2 = kM1 * x2;
    x0 = h2 ^ x1 ^ k0;
    x1 = l2;
    x2 = h0 ^ x3 ^ k1;
    x3 = l0;
  }
  const double u1 = ((double)(x0 >> 11) + 1.0) * 0x1p-53;
  const double u2 = (double)(x1 >> 11) * 0x1p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Draw index of an application: the host's value for a standalone apply,
// else the solve's count of applications so far plus the application's
// position within the current phase (start-up or iteration).
__device__ __forceinline__ unsigned long long noise_draw(const SolveState* st, long long fixed, int offset) {
  return fixed >= 0 ? (unsigned long long)fixed : st->pc.ndraws + (unsigned long long)offset;
}

// A phase (start-up, iteration) that applies B: k_noise_mark before its first
// kernel notes whether it runs at all; k_noise_advance after its last kernel
// (after the join of its streams) adds its `count` applications when the
// method went on to use them, i.e. unless the phase ended in convergence.
// The count is then that of a method that tests convergence before applying
// B, whatever the order of the concurrent reduction and preconditioner
// kernels inside the phase.
__global__ void k_noise_mark(SolveState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->pc.noise_live = read_status(st) == kRunning;
}
__global__ void k_noise_advance(SolveState* st, int count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int s = read_status(st);
  if (st->pc.noise_live && (s == kRunning || s == kBreakdown || s == kCycleEnd))
    st->pc.ndraws += (unsigned long long)count;
  st->pc.noise_live = 0;
}

// Partials of ||v||^2 and ||g||^2, v = c1 X1 + c2 X2.
__global__ void __launch_bounds__(kBlock)
k_noise_norms(long long N, const double* __restrict__ X1, double c1, const double* __restrict__ X2, double c2,
              unsigned long long seed, long long fixed, int offset, double* part, const SolveState* st) {
  if (!wg_running(st)) return;
  const unsigned long long d = noise_draw(st, fixed, offset);
  double acc[2] = {0.0, 0.0};
  for (long long e = gtid(); e < N; e += gstride()) {
    double v = c1 * X1[e];
    if (X2 != nullptr) v += c2 * X2[e];
    const double g = noise_normal(seed, d, (unsigned long long)e);
    acc[0] += v * v;
    acc[1] += g * g;
  }
  block_partials<2>(acc, 2, part, gridDim.x);
}

// y = v + (eta ||v|| / ||g||) g.
__global__ void __launch_bounds__(kBlock)
k_noise_apply(long long N, const double* __restrict__ X1, double c1, const double* __restrict__ X2, double c2,
              unsigned long long seed, long long fixed, int offset, double eta, const double* part, int P,
              double* __restrict__ y, const SolveState* st) {
  if (!wg_running(st)) return;
  const double vv = block_sum_column(part, P, 0);
  const double gg = block_sum_column(part, P, 1);
  const double s = (vv > 0.0 && gg > 0.0) ? eta * sqrt(vv) / sqrt(gg) : 0.0;
  const unsigned long long d = noise_draw(st, fixed, offset);
  for (long long e = gtid(); e < N; e += gstride()) {
    double v = c1 * X1[e];
    if (X2 != nullptr) v += c2 * X2[e];
    y[e] = v + s * noise_normal(seed, d, (unsigned long long)e);
  }
}

}  // namespace pfk
