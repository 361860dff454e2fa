// Device-side building blocks shared by every kernel of the library:
// launch geometry, the variable-coefficient stencil (one node at a time, and
// the z-marching tile engine the hot kernels use), wave/workgroup reductions
// that write per-workgroup partial sums, and the consumer-side deterministic
// reduction of those partials.
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

#include <type_traits>

namespace pfk {

constexpr int kBlock = 256;        // threads per workgroup: four 64-wide waves
constexpr int kWaves = kBlock / 64;
constexpr int kNuMax = 64;         // largest window / restart length supported

// ---------------------------------------------------------------------------
// Operator description passed by value to kernels.  C is the stored
// viscosity type, V the face-velocity type: FP64/FP64 for the operator of the
// outer iteration, BF16/FP32 for the mixed-precision inner solve.
// ---------------------------------------------------------------------------
template <class C, class V = C>
struct GridT {
  int dim, nx, ny, nz;             // interior sizes; nz == 1 for 2D
  long long N;                     // nx*ny*nz
  long long sy, sz;                // padded strides: nx+2 and (nx+2)(ny+2)
  long long vstride;               // padded node count (offset between velocity components)
  double h2inv, hinv;              // 1/h^2 and 1/h
  const C* eta;                    // padded viscosity
  const V* vel;                    // 3*vstride face velocities or nullptr
};
using Grid = GridT<double, double>;
using GridM = GridT<__hip_bfloat16, float>;

__device__ __forceinline__ double to_real(double x) { return x; }
__device__ __forceinline__ float to_real(float x) { return x; }
__device__ __forceinline__ float to_real(__hip_bfloat16 x) { return __bfloat162float(x); }

template <class G>
__device__ __forceinline__ long long padded_index(const G& g, int i, int j, int k) {
  return (g.dim == 3 ? (long long)(k + 1) * g.sz : 0) + (long long)(j + 1) * g.sy + (i + 1);
}

template <class G>
__device__ __forceinline__ long long vec_index(const G& g, int i, int j, int k) {
  return ((long long)k * g.ny + j) * g.nx + i;
}

template <class T>
__device__ __forceinline__ T harmonic(T a, T b) { return T(2) * a * b / (a + b); }

// (A u) at a node from its value uc, its six neighbour values (0 on the
// Dirichlet boundary) and the viscosities at the node and its neighbours, in
// arithmetic type T.  Diffusion: h^-2 sum_f k_f (u_c - u_nb) with k_f the
// harmonic mean of eta; convection (if the operator has face velocities):
// first-order upwind flux h^-1 sum_f (max(v_f,0) u_c + min(v_f,0) u_nb) with
// v_f the outward normal velocity.  Faces are taken in the order x+, x-, y+,
// y-, z+, z-.  The two parts are separate so that every form of the operator
// (velocities loaded here or ahead of use) rounds alike.
template <class T, class G>
__device__ __forceinline__ T faces_diffusion(const G& g, T uc, T ec, T exp_, T exm, T eyp, T eym, T ezp, T ezm,
                                             T uxp, T uxm, T uyp, T uym, T uzp, T uzm) {
  T acc = harmonic(ec, exp_) * (uc - uxp) + harmonic(ec, exm) * (uc - uxm) +
          harmonic(ec, eyp) * (uc - uyp) + harmonic(ec, eym) * (uc - uym);
  if (g.dim == 3) acc += harmonic(ec, ezp) * (uc - uzp) + harmonic(ec, ezm) * (uc - uzm);
  return acc * T(g.h2inv);
}
// The upwind sum (before the h^-1 factor) from the node's face velocities
// vx(p), vx(p - e_x), vy(p), vy(p - e_y), vz(p), vz(p - e_z).
template <class T, class G>
__device__ __forceinline__ T faces_convection(const G& g, T uc, T uxp, T uxm, T uyp, T uym, T uzp, T uzm, T vxp,
                                              T vxm, T vyp, T vym, T vzp, T vzm) {
  const T zero = T(0);
  T c = zero, v;
  v = vxp;   c += fmax(v, zero) * uc + fmin(v, zero) * uxp;
  v = -vxm;  c += fmax(v, zero) * uc + fmin(v, zero) * uxm;
  v = vyp;   c += fmax(v, zero) * uc + fmin(v, zero) * uyp;
  v = -vym;  c += fmax(v, zero) * uc + fmin(v, zero) * uym;
  if (g.dim == 3) {
    v = vzp;   c += fmax(v, zero) * uc + fmin(v, zero) * uzp;
    v = -vzm;  c += fmax(v, zero) * uc + fmin(v, zero) * uzm;
  }
  return c;
}

// The whole operator at the node with padded index pc, velocities (if any)
// loaded here.
template <class T, class G>
__device__ __forceinline__ T apply_faces(const G& g, long long pc, T uc, T ec, T exp_, T exm, T eyp, T eym,
                                         T ezp, T ezm, T uxp, T uxm, T uyp, T uym, T uzp, T uzm) {
  T acc = faces_diffusion<T>(g, uc, ec, exp_, exm, eyp, eym, ezp, ezm, uxp, uxm, uyp, uym, uzp, uzm);
  if (g.vel != nullptr) {
    const auto* vx = g.vel;
    const auto* vy = g.vel + g.vstride;
    const auto* vz = g.vel + 2 * g.vstride;
    const bool d3 = g.dim == 3;
    const T c = faces_convection<T>(g, uc, uxp, uxm, uyp, uym, uzp, uzm, T(to_real(vx[pc])),
                                    T(to_real(vx[pc - 1])), T(to_real(vy[pc])), T(to_real(vy[pc - g.sy])),
                                    d3 ? T(to_real(vz[pc])) : T(0), d3 ? T(to_real(vz[pc - g.sz])) : T(0));
    acc += T(g.hinv) * c;
  }
  return acc;
}

// (A u) at interior node (i,j,k), flat index idx, one node at a time, FP64:
// U is an accessor for interior neighbour values.
template <class F>
__device__ __forceinline__ double stencil_at(const Grid& g, int i, int j, int k, long long idx,
                                             double uc, F&& U) {
  const long long pc = padded_index(g, i, j, k);
  const long long nxy = (long long)g.nx * g.ny;
  const bool d3 = g.dim == 3;
  return apply_faces<double>(g, pc, uc, g.eta[pc], g.eta[pc + 1], g.eta[pc - 1], g.eta[pc + g.sy],
                             g.eta[pc - g.sy], d3 ? g.eta[pc + g.sz] : 0.0, d3 ? g.eta[pc - g.sz] : 0.0,
                             (i + 1 < g.nx) ? U(idx + 1) : 0.0, (i > 0) ? U(idx - 1) : 0.0,
                             (j + 1 < g.ny) ? U(idx + g.nx) : 0.0, (j > 0) ? U(idx - g.nx) : 0.0,
                             (d3 && k + 1 < g.nz) ? U(idx + nxy) : 0.0, (d3 && k > 0) ? U(idx - nxy) : 0.0);
}

// Stencil launch geometry.  A workgroup owns a tile of x-y nodes, 64 x 8 or
// 32 x 16 (two rows per thread either way), and walks `zc` consecutive
// z-planes, so the number of workgroups (and of reduction partials) is
// tiles_x * tiles_y * ceil(nz/zc).  The tile width is per operator: narrow
// grids (n = 32, 96, ...) waste fewer lanes on 32-wide tiles.
struct StencilGeom {
  int tiles_x, tiles_y, zc, zchunks;
  int tx;                                   // tile width: 64 or 32
  __host__ __device__ int blocks() const { return tiles_x * tiles_y * zchunks; }
};

template <int TX>
struct TileShape {
  static constexpr int TY = 2 * kBlock / TX;       // tile rows: 8 or 16
  static constexpr int RPW = 64 / TX;              // rows one wave covers in a pass
  static constexpr int HALO = 2 * TX + 2 * TY;     // in-plane halo nodes
  static_assert(HALO <= kBlock, "one halo node per thread at most");
};

// Workgroup ids are dealt round-robin to the 8 XCDs (each with its own L2).
// Give each XCD a contiguous run of tiles (x fastest, then y, then z-chunk)
// so the halo rows and planes that neighbouring tiles share stay in one L2.
// b is the workgroup's index within its launch (or within its system's range
// of a batched launch, which starts at a multiple of 8).
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int full = nblocks & ~7;
  if (b >= full) return b;
  return (b & 7) * (full >> 3) + (b >> 3);
}
__device__ __forceinline__ int xcd_tile(int nblocks) { return xcd_tile(blockIdx.x, nblocks); }

// Iterate the nodes a workgroup owns in a stencil launch (one node at a time).
template <int TX, class G, class F>
__device__ __forceinline__ void for_tile_nodes_t(const G& g, const StencilGeom& sg, int bid, F&& body) {
  using S = TileShape<TX>;
  const int L = xcd_tile(bid, sg.blocks());
  const int tx = L % sg.tiles_x;
  const int ty = (L / sg.tiles_x) % sg.tiles_y;
  const int tz = L / (sg.tiles_x * sg.tiles_y);
  const int lane = threadIdx.x & 63;
  const int i = tx * TX + lane % TX;
  const int r0 = (threadIdx.x >> 6) * S::RPW + lane / TX;
  const int k0 = tz * sg.zc;
  const int k1 = min(g.nz, k0 + sg.zc);
  for (int r = 0; r < 2; ++r) {
    const int j = ty * S::TY + r0 + r * (S::TY / 2);
    if (i >= g.nx || j >= g.ny) continue;
    for (int k = k0; k < k1; ++k) body(i, j, k, vec_index(g, i, j, k));
  }
}
template <class G, class F>
__device__ __forceinline__ void for_tile_nodes(const G& g, const StencilGeom& sg, F&& body) {
  if (sg.tx == 32) for_tile_nodes_t<32>(g, sg, blockIdx.x, body);
  else for_tile_nodes_t<64>(g, sg, blockIdx.x, body);
}

// Nontemporal element access for kernels that stream vectors much larger
// than the caches.
template <class T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void stnt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Input of the stencil engine: load(t) issues the global loads of flat node t
// and nothing else (its result is a value, or a struct of loaded values);
// value(raw) forms the node's input u from them.  The engine issues loads
// ahead and forms values only when their plane is reached, so no arithmetic
// on loaded data makes a plane step wait for its own prefetch.  keep(t, raw,
// slot) is called once for every node the workgroup owns (never for its
// halo), with the raw loads its value is formed from: a caller that also
// stores a value derived from the input (the next inner basis vector, say)
// does it there.  slot = 2 (plane & 1) + row names the node among the
// thread's own nodes of two consecutive planes; a node is kept two plane
// steps before its sink call, and a sink that takes a fourth argument gets
// the same slot, so a caller can hand per-node data from keep to sink
// through thread-private storage of four entries.
struct NoKeep {
  template <class R>
  __device__ __forceinline__ void operator()(long long, const R&, int) const {}
};
template <class LoadF, class ValueF, class KeepF = NoKeep>
struct StencilIn {
  LoadF load;
  ValueF value;
  KeepF keep;
};
template <class LoadF, class ValueF>
__device__ __forceinline__ StencilIn<LoadF, ValueF> stencil_in(LoadF load, ValueF value) {
  return StencilIn<LoadF, ValueF>{load, value, NoKeep{}};
}
template <class LoadF, class ValueF, class KeepF>
__device__ __forceinline__ StencilIn<LoadF, ValueF, KeepF> stencil_in(LoadF load, ValueF value, KeepF keep) {
  return StencilIn<LoadF, ValueF, KeepF>{load, value, keep};
}
// An input formed where it is loaded (a plain load, or a combination the
// caller evaluates at once).
template <class LoadF>
__device__ __forceinline__ auto stencil_in(LoadF load) {
  return stencil_in(load, [](auto v) { return v; });
}

// The hot stencil engine, in arithmetic type T.  A workgroup walks its tile
// up the z-axis.  Each node's input value u = in.value(in.load(flat index)) is
// formed once.
// z-neighbours stay in registers; in-plane neighbours of u and of the
// viscosity come from LDS copies of the plane with a one-node halo (halo
// values are formed by the first 2(TX+TY) threads).  Loads run PD plane
// steps ahead: while plane k is computed, the loads of planes k+2 .. k+1+PD
// are in flight, for the centre column and for the halo alike.  A tile's halo
// rows are interior rows of its neighbours, which those load in the same
// plane step, so the second request finds the line in (or on its way into)
// the XCD's L2 instead of fetching it again from HBM.  At the end of step k
// the values of plane k+2 are formed: the column's into registers, the
// halo's straight into the LDS buffer of their plane (three plane buffers in
// a ring: k being read, k+1 complete, k+2 receiving its halo), so no formed
// halo value is held in a register across a step.  PD = 1 waits at the end
// of a step for loads issued at its start; PD = 2 keeps a second plane of raw
// loads in registers and waits for loads a whole step old -- worth it where
// the extra registers cost no occupancy step (the FP32 inner GMRES apply at
// 256^3: 0.160 -> 0.133 ms), not where they do (the FP64 inner PCG kernels
// lose one and slow down 3-10%).  Values outside the domain are 0
// (Dirichlet); viscosities are read on the whole padded grid.
// For every interior node the engine calls sink(flat index, u, (A u)).
//
// LDS of the stencil engine: kStencilSlots plane buffers of u and of the
// viscosity, sized for the larger tile (64x8 and 32x16 tiles with their
// halo); one buffer per word size, shared by every tile width and caller of
// that size -- a static in a function is a single object per instantiation,
// so a kernel holds it once however many variants it uses.
constexpr int kStencilSlots = 3;
constexpr int kStencilPlane = (TileShape<64>::TY + 2) * (64 + 2);
static_assert(kStencilPlane >= (TileShape<32>::TY + 2) * (32 + 2), "LDS sized for the larger tile");
template <int B>
__device__ __forceinline__ char* stencil_lds() {
  __shared__ __attribute__((aligned(16))) char buf[kStencilSlots * 2 * kStencilPlane * B];
  return buf;
}

// CV: how the face velocities of a convective operator are loaded.
// 0: where they are used (apply_faces; any operator), 1: one plane step
// ahead into registers like the column's u and eta, 2: at the start of their
// own plane step, so they are in flight during the step's barriers and LDS
// exchange -- for kernels whose registers leave no room for a second plane of
// velocities.  With 1 and 2 the z- face of a plane is the z+ face of the one
// below, kept from the previous step.  CV kernels are separate
// instantiations, so the diffusion kernels do not carry the extra registers.
template <int TX, int CV, int PD, class T, class G, class In, class Sink>
__device__ __forceinline__ void stencil_march_t(const G& g, const StencilGeom& sg, int bid, const In& in,
                                                Sink& sink) {
  static_assert(PD >= 1 && PD <= 3, "prefetch depth 1..3 plane steps");
  using S = TileShape<TX>;
  constexpr int TY = S::TY;
  constexpr int PL = (TY + 2) * (TX + 2);
  T* const lds = reinterpret_cast<T*>(stencil_lds<sizeof(T)>());
  // plane buffer of ring slot s: u at lds + 2 s PL, the viscosity after it
  auto SU = [&](int s) { return reinterpret_cast<T (*)[TX + 2]>(lds + 2 * s * PL); };
  auto SE = [&](int s) { return reinterpret_cast<T (*)[TX + 2]>(lds + (2 * s + 1) * PL); };
  const int L = xcd_tile(bid, sg.blocks());
  const int tx = L % sg.tiles_x;
  const int ty = (L / sg.tiles_x) % sg.tiles_y;
  const int tz = L / (sg.tiles_x * sg.tiles_y);
  const int lane = threadIdx.x & 63;
  const int xo = lane % TX;
  const int r0 = (threadIdx.x >> 6) * S::RPW + lane / TX;
  const int i0 = tx * TX, j0 = ty * TY;
  const int i = i0 + xo;
  const int k0 = tz * sg.zc;
  const int k1 = min(g.nz, k0 + sg.zc);
  const bool d3 = g.dim == 3;
  const int kmax = d3 ? g.nz : 0;          // last padded z-plane index minus 1
  const T zero = T(0);
  int jr[2], row[2];
  bool valid[2], evalid[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    row[r] = r0 + r * (TY / 2);
    jr[r] = j0 + row[r];
    valid[r] = i < g.nx && jr[r] < g.ny;
    evalid[r] = i <= g.nx && jr[r] <= g.ny;   // on the padded grid (boundary ring included)
  }
  // this thread's halo node (if any) and its LDS slot
  const int t = threadIdx.x;
  int hi = 0, hj = 0, hr = 0, hc = 0;
  if (t < TX) { hi = i0 + t; hj = j0 - 1; hr = 0; hc = t + 1; }
  else if (t < 2 * TX) { hi = i0 + t - TX; hj = j0 + TY; hr = TY + 1; hc = t - TX + 1; }
  else if (t < 2 * TX + TY) { hi = i0 - 1; hj = j0 + t - 2 * TX; hr = hj - j0 + 1; hc = 0; }
  else if (t < S::HALO) { hi = i0 + TX; hj = j0 + t - 2 * TX - TY; hr = hj - j0 + 1; hc = TX + 1; }
  const bool has_halo = t < S::HALO;
  const bool hvalid = has_halo && hi >= 0 && hi < g.nx && hj >= 0 && hj < g.ny;
  const bool hevalid = has_halo && hi >= -1 && hi <= g.nx && hj >= -1 && hj <= g.ny;

  // raw loads (R suffix) and the values formed from them
  using Raw = decltype(in.load(0LL));
  using ES = typename std::remove_cv<typename std::remove_pointer<decltype(g.eta)>::type>::type;
  const ES ez = ES(0.0f);
  auto UOK = [&](int r, int k) { return valid[r] && k >= 0 && k < g.nz; };
  auto UR = [&](int r, int k) { return UOK(r, k) ? in.load(vec_index(g, i, jr[r], k)) : Raw{}; };
  auto U = [&](int r, int k) { return UOK(r, k) ? T(in.value(UR(r, k))) : zero; };
  auto ER = [&](int r, int k) {
    return (evalid[r] && k >= -1 && k <= kmax) ? g.eta[padded_index(g, i, jr[r], k)] : ez;
  };
  auto E = [&](int r, int k) { return T(to_real(ER(r, k))); };
  auto HOK = [&](int k) { return hvalid && k < g.nz; };
  auto HER = [&](int k) { return (hevalid && k <= kmax) ? g.eta[padded_index(g, hi, hj, k)] : ez; };

  // a previous march of this workgroup may still be reading the buffers
  __syncthreads();
  // register window: m = k-1, c = k, p = k+1 (u and eta of the centre column)
  T um[2], uc[2], up[2], em[2], ec[2], ep[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    um[r] = d3 ? U(r, k0 - 1) : zero;
    uc[r] = zero;
    if (k0 < k1 && UOK(r, k0)) {
      const long long t0 = vec_index(g, i, jr[r], k0);
      const Raw q = in.load(t0);
      uc[r] = T(in.value(q));
      in.keep(t0, q, ((k0 & 1) << 1) | r);
    }
    up[r] = zero;
    if (d3 && UOK(r, k0 + 1)) {
      const long long t1 = vec_index(g, i, jr[r], k0 + 1);
      const Raw q = in.load(t1);
      up[r] = T(in.value(q));
      if (k0 + 1 < k1) in.keep(t1, q, (((k0 + 1) & 1) << 1) | r);
    }
    em[r] = d3 ? E(r, k0 - 1) : zero;
    ec[r] = E(r, k0);
    ep[r] = d3 ? E(r, k0 + 1) : zero;
  }
  // halo of planes k0 and k0+1 into ring slots 0 and 1
  if (has_halo) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int kk = k0 + d;
      if (kk < k1) {
        SU(d)[hr][hc] = HOK(kk) ? T(in.value(in.load(vec_index(g, hi, hj, kk)))) : zero;
        SE(d)[hr][hc] = T(to_real(HER(kk)));
      }
    }
  }
  // raw loads of one plane p: the column's (needed while plane p-1 is
  // computed, i.e. if p-1 < k1) and the halo's (needed if p < k1)
  struct ColRaw {
    Raw u[2];
    ES e[2];
    bool ok[2];
  };
  struct HaloRaw {
    Raw u;
    ES e;
    bool h, ok;
  };
  auto issue_col = [&](int p) {
    ColRaw c;
    const bool need = d3 && p - 1 < k1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      c.ok[r] = need && UOK(r, p);
      c.u[r] = c.ok[r] ? in.load(vec_index(g, i, jr[r], p)) : Raw{};
      c.e[r] = need ? ER(r, p) : ez;
    }
    return c;
  };
  auto issue_halo = [&](int p) {
    HaloRaw h;
    h.h = has_halo && p < k1;
    h.ok = h.h && HOK(p);
    h.u = h.ok ? in.load(vec_index(g, hi, hj, p)) : Raw{};
    h.e = h.h ? HER(p) : ez;
    return h;
  };
  // planes k0+2 .. k0+PD in flight before the first step (PD > 1)
  ColRaw cq[PD > 1 ? PD - 1 : 1];
  HaloRaw hq[PD > 1 ? PD - 1 : 1];
  if constexpr (PD > 1) {
#pragma unroll
    for (int d = 0; d < PD - 1; ++d) {
      cq[d] = issue_col(k0 + 2 + d);
      hq[d] = issue_halo(k0 + 2 + d);
    }
  }
  int slot = 0;   // ring slot of plane k
  // face velocities of the centre column (CV): x+, x-, y+, y-, z+ of the
  // current plane, of the next one in flight, and z- of the current plane
  T vc[2][5], vn[2][5], vzm[2];
  auto VL = [&](int r, int k, T (&v)[5]) {
    const T zero_ = T(0);
#pragma unroll
    for (int f = 0; f < 5; ++f) v[f] = zero_;
    if (valid[r]) {
      const long long pc = padded_index(g, i, jr[r], k);
      v[0] = T(to_real(g.vel[pc]));
      v[1] = T(to_real(g.vel[pc - 1]));
      v[2] = T(to_real(g.vel[g.vstride + pc]));
      v[3] = T(to_real(g.vel[g.vstride + pc - g.sy]));
      if (d3) v[4] = T(to_real(g.vel[2 * g.vstride + pc]));
    }
  };
  if constexpr (CV != 0) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (CV == 1 && k0 < k1) VL(r, k0, vc[r]);
      vzm[r] = (d3 && valid[r] && k0 < k1) ? T(to_real(g.vel[2 * g.vstride + padded_index(g, i, jr[r], k0) - g.sz]))
                                           : zero;
    }
  }
  for (int k = k0; k < k1; ++k) {
    // issued this step: plane k+1+PD of the column and of the halo
    const ColRaw cn = issue_col(k + 1 + PD);
    const HaloRaw hn = issue_halo(k + 1 + PD);
    const bool more = k + 1 < k1;
    if constexpr (CV == 1) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (more) VL(r, k + 1, vn[r]);
      }
    } else if constexpr (CV == 2) {
#pragma unroll
      for (int r = 0; r < 2; ++r) VL(r, k, vc[r]);
    }
    T (*const su)[TX + 2] = SU(slot);
    T (*const se)[TX + 2] = SE(slot);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      su[row[r] + 1][xo + 1] = uc[r];
      se[row[r] + 1][xo + 1] = ec[r];
    }
    __syncthreads();
    // the raw loads of plane k+2, formed at the end of this step
    const ColRaw& c2 = PD > 1 ? cq[0] : cn;
    const HaloRaw& h2 = PD > 1 ? hq[0] : hn;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (valid[r]) {
        const int rr = row[r] + 1;
        T Au;
        if constexpr (CV != 0) {
          const T uxp = su[rr][xo + 2], uxm = su[rr][xo], uyp = su[rr + 1][xo + 1], uym = su[rr - 1][xo + 1];
          Au = faces_diffusion<T>(g, uc[r], ec[r], se[rr][xo + 2], se[rr][xo], se[rr + 1][xo + 1],
                                  se[rr - 1][xo + 1], ep[r], em[r], uxp, uxm, uyp, uym, up[r], um[r]);
          Au += T(g.hinv) * faces_convection<T>(g, uc[r], uxp, uxm, uyp, uym, up[r], um[r], vc[r][0], vc[r][1],
                                                vc[r][2], vc[r][3], vc[r][4], vzm[r]);
        } else {
          const long long pc = padded_index(g, i, jr[r], k);
          Au = apply_faces<T>(g, pc, uc[r], ec[r], se[rr][xo + 2], se[rr][xo], se[rr + 1][xo + 1],
                              se[rr - 1][xo + 1], ep[r], em[r], su[rr][xo + 2], su[rr][xo], su[rr + 1][xo + 1],
                              su[rr - 1][xo + 1], up[r], um[r]);
        }
        if constexpr (std::is_invocable_v<Sink&, long long, T, T, int>)
          sink(vec_index(g, i, jr[r], k), uc[r], Au, ((k & 1) << 1) | r);
        else
          sink(vec_index(g, i, jr[r], k), uc[r], Au);
      }
      if constexpr (CV != 0) vzm[r] = vc[r][4];
      if constexpr (CV == 1) {
#pragma unroll
        for (int f = 0; f < 5; ++f) vc[r][f] = vn[r][f];
      }
      um[r] = uc[r];
      uc[r] = up[r];
      up[r] = c2.ok[r] ? T(in.value(c2.u[r])) : zero;
      if (c2.ok[r] && k + 2 < k1) in.keep(vec_index(g, i, jr[r], k + 2), c2.u[r], ((k & 1) << 1) | r);
      em[r] = ec[r];
      ec[r] = ep[r];
      ep[r] = T(to_real(c2.e[r]));
    }
    // the halo of plane k+2 into the slot plane k-1 used (every thread has
    // passed this step's barriers, so none still reads it)
    const int s2 = slot == 0 ? kStencilSlots - 1 : slot - 1;
    if (h2.h) {
      SU(s2)[hr][hc] = h2.ok ? T(in.value(h2.u)) : zero;
      SE(s2)[hr][hc] = T(to_real(h2.e));
    }
    if constexpr (PD > 1) {
#pragma unroll
      for (int d = 0; d + 1 < PD - 1; ++d) {
        cq[d] = cq[d + 1];
        hq[d] = hq[d + 1];
      }
      cq[PD - 2] = cn;
      hq[PD - 2] = hn;
    }
    slot = slot == kStencilSlots - 1 ? 0 : slot + 1;
  }
}

template <class T, int CV = 0, int PD = 1, class G, class In, class Sink>
__device__ __forceinline__ void stencil_march(const G& g, const StencilGeom& sg, int bid, const In& in, Sink& sink) {
  if (sg.tx == 32) stencil_march_t<32, CV, PD, T>(g, sg, bid, in, sink);
  else stencil_march_t<64, CV, PD, T>(g, sg, bid, in, sink);
}
template <class T, int CV = 0, int PD = 1, class G, class In, class Sink>
__device__ __forceinline__ void stencil_march(const G& g, const StencilGeom& sg, const In& in, Sink& sink) {
  stencil_march<T, CV, PD>(g, sg, (int)blockIdx.x, in, sink);
}

// ---------------------------------------------------------------------------
// Reductions.  Every reducing kernel writes, per workgroup b and column c,
// part[c * P + b] (P = number of workgroups).  The sums over b are taken in
// a fixed order by the consumer, so results are deterministic run to run.
// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a wave, the same value in every lane: an
// inclusive scan within each row of 16 lanes (DPP row shifts by 1, 2, 4, 8),
// the row totals carried across rows (row broadcasts of lanes 15 and 31),
// then lane 63's total read into a scalar.  DPP moves data between lanes in
// the VALU; a shuffle would go through the LDS crossbar (two permutes per
// step for a double): in the window update, which sums a dot per window
// direction, the shuffle form cost about 1.3% of the kernel's time.
// Lanes outside a row's shift range contribute 0 (bound_ctrl), rows outside
// a broadcast's row mask keep their value.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0x111, 0xf>(v);   // row_shr:1
  v += dpp_mov<0x112, 0xf>(v);   // row_shr:2
  v += dpp_mov<0x114, 0xf>(v);   // row_shr:4
  v += dpp_mov<0x118, 0xf>(v);   // row_shr:8
  v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum NC per-thread accumulators over the workgroup; column c of workgroup
// blockIdx.x goes to part[c*P + blockIdx.x] for c < nc.  Every thread of the
// workgroup must call this (it synchronises).
template <int NC>
__device__ __forceinline__ void block_partials(double (&acc)[NC], int nc, double* part, int P, int bid) {
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
    part[(long long)c * P + bid] = s;
  }
}
template <int NC>
__device__ __forceinline__ void block_partials(double (&acc)[NC], int nc, double* part, int P) {
  block_partials<NC>(acc, nc, part, P, (int)blockIdx.x);
}

// Sum column c of P partials with the whole workgroup (fixed order); the
// result is returned to every thread.  Every thread must call this.  Eight
// independent partial sums per thread keep eight loads in flight (a kernel's
// prologue reads up to 16384 partials of the previous launch).
__device__ __forceinline__ double block_sum_column(const double* part, int P, int c) {
  __shared__ double sh[kWaves];
  __shared__ double result;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double* col = part + (long long)c * P;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 7 * kBlock < P; b += 8 * kBlock) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] += col[b + q * kBlock];
  }
  for (; b < P; b += kBlock) a[0] += col[b];
  double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
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

// Sum columns 0..ncol-1 of P partials into out[] (shared memory), one wave
// per column in turn, fixed order.  Every thread must call this; out[] is
// valid for all threads on return.
__device__ __forceinline__ void block_sum_columns(const double* part, int P, int ncol, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = wid; c < ncol; c += kWaves) {
    // eight independent partial sums per lane keep eight loads in flight
    const double* col = part + (long long)c * P;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = lane;
    for (; b + 7 * 64 < P; b += 8 * 64) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += col[b + q * 64];
    }
    for (; b < P; b += 64) a[0] += col[b];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = wave_sum(s);
    if (lane == 0) out[c] = s;
  }
  __syncthreads();
}

// A workgroup's place in its launch.  A single-system kernel is a launch of
// its own (id = blockIdx.x, n = gridDim.x); a batched kernel gives every
// system its own contiguous range of workgroups.
struct Blk {
  int id, n;
  __device__ __forceinline__ long long gtid() const { return (long long)id * kBlock + threadIdx.x; }
  __device__ __forceinline__ long long gstride() const { return (long long)n * kBlock; }
};
__device__ __forceinline__ Blk this_blk() { return Blk{(int)blockIdx.x, (int)gridDim.x}; }

// Grid-stride geometry for pointwise kernels.
__device__ __forceinline__ long long gtid() { return (long long)blockIdx.x * kBlock + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * kBlock; }

}  // namespace pfk
