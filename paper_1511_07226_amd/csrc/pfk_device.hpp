// Device-side building blocks shared by every kernel of the library:
// launch geometry, the variable-coefficient stencil evaluated at one node,
// wave/workgroup reductions that write per-workgroup partial sums, and the
// consumer-side deterministic reduction of those partials.
//
// Layout conventions (the same as the C ABI):
//   * unknown vectors: N = nx*ny*nz FP64 values (nz = 1 in 2D), x fastest;
//   * eta: node viscosity on the padded grid (nx+2)(ny+2)(nz+2), x fastest
//     (2D: (nx+2)(ny+2)); padded index 0 and n+1 are the Dirichlet boundary;
//   * face velocities: three padded arrays (x, y, z components); component c
//     at padded node p is the velocity on the face between p and p + e_c.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace pfk {

constexpr int kBlock = 256;        // threads per workgroup: four 64-wide waves
constexpr int kWaves = kBlock / 64;
constexpr int kTileX = 64;         // stencil tile: 64 x-nodes (one wave per row) ...
constexpr int kTileY = 4;          // ... by 4 y-rows
constexpr int kNuMax = 64;         // largest window / restart length supported

// ---------------------------------------------------------------------------
// Operator description passed by value to kernels.
// ---------------------------------------------------------------------------
template <class C>
struct GridT {
  int dim, nx, ny, nz;             // interior sizes; nz == 1 for 2D
  long long N;                     // nx*ny*nz
  long long sy, sz;                // padded strides: nx+2 and (nx+2)(ny+2)
  long long vstride;               // padded node count (offset between velocity components)
  double h2inv, hinv;              // 1/h^2 and 1/h
  const C* eta;                    // padded viscosity (FP64, or BF16 for the mixed inner solve)
  const C* vel;                    // 3*vstride face velocities or nullptr
};
using Grid = GridT<double>;

__device__ __forceinline__ long long padded_index(const Grid& g, int i, int j, int k) {
  return (g.dim == 3 ? (long long)(k + 1) * g.sz : 0) + (long long)(j + 1) * g.sy + (i + 1);
}

__device__ __forceinline__ double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

// (A u) at interior node (i,j,k), flat index idx, given u at the node (uc) and
// an accessor U(flat index) for its interior neighbours.  Diffusion:
// h^-2 sum_f k_f (u_c - u_nb), k_f the harmonic mean of eta; Dirichlet
// neighbours contribute u_nb = 0.  Convection (if g.vel): first-order upwind
// flux h^-1 sum_f (max(v_f,0) u_c + min(v_f,0) u_nb) with outward v_f.
template <class F>
__device__ __forceinline__ double stencil_at(const Grid& g, int i, int j, int k, long long idx,
                                             double uc, F&& U) {
  const long long pc = padded_index(g, i, j, k);
  const double ec = g.eta[pc];
  const double un_xp = (i + 1 < g.nx) ? U(idx + 1) : 0.0;
  const double un_xm = (i > 0) ? U(idx - 1) : 0.0;
  const double un_yp = (j + 1 < g.ny) ? U(idx + g.nx) : 0.0;
  const double un_ym = (j > 0) ? U(idx - g.nx) : 0.0;
  double acc = harmonic(ec, g.eta[pc + 1]) * (uc - un_xp) + harmonic(ec, g.eta[pc - 1]) * (uc - un_xm) +
               harmonic(ec, g.eta[pc + g.sy]) * (uc - un_yp) + harmonic(ec, g.eta[pc - g.sy]) * (uc - un_ym);
  double un_zp = 0.0, un_zm = 0.0;
  if (g.dim == 3) {
    const long long nxy = (long long)g.nx * g.ny;
    un_zp = (k + 1 < g.nz) ? U(idx + nxy) : 0.0;
    un_zm = (k > 0) ? U(idx - nxy) : 0.0;
    acc += harmonic(ec, g.eta[pc + g.sz]) * (uc - un_zp) + harmonic(ec, g.eta[pc - g.sz]) * (uc - un_zm);
  }
  acc *= g.h2inv;
  if (g.vel != nullptr) {
    const double* vx = g.vel;
    const double* vy = g.vel + g.vstride;
    const double* vz = g.vel + 2 * g.vstride;
    double c = 0.0, v;
    v = vx[pc];            c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_xp;
    v = -vx[pc - 1];       c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_xm;
    v = vy[pc];            c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_yp;
    v = -vy[pc - g.sy];    c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_ym;
    if (g.dim == 3) {
      v = vz[pc];          c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_zp;
      v = -vz[pc - g.sz];  c += fmax(v, 0.0) * uc + fmin(v, 0.0) * un_zm;
    }
    acc += g.hinv * c;
  }
  return acc;
}

// Stencil launch geometry: a workgroup owns a 64 x 4 tile of x-y nodes and
// walks `zc` consecutive z-planes, so the number of workgroups (and of
// reduction partials) is tiles_x * tiles_y * ceil(nz/zc).
struct StencilGeom {
  int tiles_x, tiles_y, zc, zchunks;
  __host__ __device__ int blocks() const { return tiles_x * tiles_y * zchunks; }
};

// Iterate the nodes a workgroup owns in a stencil launch.
template <class F>
__device__ __forceinline__ void for_tile_nodes(const Grid& g, const StencilGeom& sg, F&& body) {
  const int b = blockIdx.x;
  const int tx = b % sg.tiles_x;
  const int ty = (b / sg.tiles_x) % sg.tiles_y;
  const int tz = b / (sg.tiles_x * sg.tiles_y);
  const int i = tx * kTileX + (threadIdx.x & 63);
  const int j = ty * kTileY + (threadIdx.x >> 6);
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = tz * sg.zc;
  const int k1 = min(g.nz, k0 + sg.zc);
  for (int k = k0; k < k1; ++k) {
    const long long idx = ((long long)k * g.ny + j) * g.nx + i;
    body(i, j, k, idx);
  }
}

// ---------------------------------------------------------------------------
// Reductions.  Every reducing kernel writes, per workgroup b and column c,
// part[c * P + b] (P = number of workgroups).  The sums over b are taken in
// a fixed order by the consumer, so results are deterministic run to run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum NC per-thread accumulators over the workgroup; column c of workgroup
// blockIdx.x goes to part[c*P + blockIdx.x] for c < nc.  Every thread of the
// workgroup must call this (it synchronises).
template <int NC>
__device__ __forceinline__ void block_partials(double (&acc)[NC], int nc, double* part, int P) {
  __shared__ double sh[kWaves][NC];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c < nc) {
      const double s = wave_sum(acc[c]);
      if (lane == 0) sh[wid][c] = s;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += kBlock) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += sh[w][c];
    part[(long long)c * P + blockIdx.x] = s;
  }
}

// Sum column c of P partials with the whole workgroup (fixed order); the
// result is returned to every thread.  Every thread must call this.
__device__ __forceinline__ double block_sum_column(const double* part, int P, int c) {
  __shared__ double sh[kWaves];
  __shared__ double result;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double s = 0.0;
  for (int b = threadIdx.x; b < P; b += kBlock) s += part[(long long)c * P + b];
  s = wave_sum(s);
  if (lane == 0) sh[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += sh[w];
    result = t;
  }
  __syncthreads();
  const double r = result;
  __syncthreads();
  return r;
}

// Grid-stride geometry for pointwise kernels.
__device__ __forceinline__ long long gtid() { return (long long)blockIdx.x * kBlock + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * kBlock; }

}  // namespace pfk
