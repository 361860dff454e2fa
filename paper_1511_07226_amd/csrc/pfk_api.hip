// C ABI of libpfk (see include/pfk.h): operators, preconditioners, sessions
// and the host driver that enqueues the kernels of one solve on two HIP
// streams, captured into hipGraphs.
//
// Stream plan of one pipelined iteration (PIPEFCG):
//
//   s1: update(j) --fork--> PC kernels (v = w - r) --> m = u + B(v), n = A m --join--> update(j+1)
//   s2:             \-----> reduction finish + scalar recurrences -----------/
//
// The reduction of iteration j+1 is produced by update(j) as per-workgroup
// partial sums; finishing it (and computing beta, eta, alpha, the test) runs
// on s2 while s1 applies B and A -- the single-GPU form of the paper's
// non-blocking all-reduce overlapped with the preconditioner and operator.
// The unpipelined methods run the same kernels in one stream with each
// reduction consumed right after it is produced.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pfk.h"
#include "pfk_batch.hpp"
#include "pfk_noise.hpp"

using namespace pfk;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PFK_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

extern "C" const char* pfk_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// helper kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_dinv(Grid g, StencilGeom sg, double* __restrict__ dinv) {
  // D_ii is the stencil applied to the unit vector at i, read at i.
  auto Z = [&](long long) { return 0.0; };
  for_tile_nodes(g, sg, [&](int i, int j, int k, long long idx) {
    dinv[idx] = 1.0 / stencil_at(g, i, j, k, idx, 1.0, Z);
  });
}

// D^-1 of the mixed-precision inner operator (BF16 eta, FP32 velocities),
// in FP32: the inner stencil applied to the unit vector at i.
__global__ void __launch_bounds__(kBlock)
k_dinv_mixed(GridM g, StencilGeom sg, float* __restrict__ dinv) {
  for_tile_nodes(g, sg, [&](int i, int j, int k, long long idx) {
    const long long pc = padded_index(g, i, j, k);
    const bool d3 = g.dim == 3;
    auto E = [&](long long q) { return to_real(g.eta[q]); };
    const float d = apply_faces<float>(g, pc, 1.0f, E(pc), E(pc + 1), E(pc - 1), E(pc + g.sy), E(pc - g.sy),
                                       d3 ? E(pc + g.sz) : 0.0f, d3 ? E(pc - g.sz) : 0.0f, 0.f, 0.f, 0.f, 0.f,
                                       0.f, 0.f);
    dinv[idx] = 1.0f / d;
  });
}

__global__ void __launch_bounds__(kBlock)
k_dot(long long N, const double* __restrict__ a, const double* __restrict__ b, double* part) {
  double acc[1] = {0.0};
  for (long long e = gtid(); e < N; e += gstride()) acc[0] += a[e] * b[e];
  block_partials<1>(acc, 1, part, gridDim.x);
}

// tol = rtol*||b||; with b = 0 the solve is finished (x is zeroed separately).
__global__ void __launch_bounds__(kBlock)
k_setup_tol(const double* part, int P, double rtol, SolveState* st, double* hist) {
  const double bb = block_sum_column(part, P, 0);
  if (threadIdx.x != 0) return;
  st->bnorm = sqrt(bb);
  st->rtol = rtol;
  st->tol = rtol * st->bnorm;
  if (bb == 0.0) {
    st->bzero = 1;
    st->status = kDone;
    hist[0] = 0.0;
    st->hist_started = 1;
  }
}

__global__ void __launch_bounds__(kBlock)
k_zero_if_done(long long N, double* __restrict__ x, const SolveState* st) {
  if (!st->bzero) return;
  for (long long e = gtid(); e < N; e += gstride()) x[e] = 0.0;
}

__global__ void __launch_bounds__(kBlock)
k_pc_write(long long N, PcOutDesc pd, double* __restrict__ y, SolveState* st) {
  if (!wg_running(st)) return;
  const PcOut pc = make_pc_out(pd, &st->pc);
  for (long long e = gtid(); e < N; e += gstride()) y[e] = pc(e);
}

// Test hook: one wave sleeps `rounds` times (s_sleep 127 each), a fixed,
// bounded delay on the stream it is launched on.
__global__ void k_delay(int rounds) {
  for (int r = 0; r < rounds; ++r) __builtin_amdgcn_s_sleep(127);
}

__global__ void k_set_running(SolveState* st, int nt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->status = kRunning;
    st->pc.ndraws = 0;
    st->nt = nt;
  }
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct pfk_operator_s {
  int dim = 0;
  int64_t n[3] = {1, 1, 1};
  long long N = 0;
  double h = 0.0;
  double* eta = nullptr;   // padded
  double* vel = nullptr;   // 3 * padded or null
  double* dinv = nullptr;  // N
  long long npad = 0;
  StencilGeom sg{};
  int pv_blocks = 0;       // workgroups of pointwise kernels
  int stencil_target = 2048;  // the workgroup target sg was made for
  // mixed-precision inner operator (made when a mixed preconditioner is created)
  __hip_bfloat16* eta_bf16 = nullptr;
  float* vel_f32 = nullptr;
  float* dinv_f32 = nullptr;

  GridM grid_mixed() const {
    GridM g;
    const Grid d = grid();
    g.dim = d.dim; g.nx = d.nx; g.ny = d.ny; g.nz = d.nz; g.N = d.N; g.sy = d.sy; g.sz = d.sz;
    g.vstride = d.vstride; g.h2inv = d.h2inv; g.hinv = d.hinv;
    g.eta = eta_bf16;
    g.vel = vel ? vel_f32 : nullptr;
    return g;
  }

  Grid grid() const {
    Grid g;
    g.dim = dim;
    g.nx = (int)n[0];
    g.ny = (int)n[1];
    g.nz = dim == 3 ? (int)n[2] : 1;
    g.N = N;
    g.sy = n[0] + 2;
    g.sz = (n[0] + 2) * (n[1] + 2);
    g.vstride = npad;
    g.h2inv = 1.0 / (h * h);
    g.hinv = 1.0 / h;
    g.eta = eta;
    g.vel = vel;
    return g;
  }
};

struct pfk_precond_s {
  pfk_operator A = nullptr;
  int kind = 0;
  int k = 1;
  int prec = 0;
  int block = 8;
  double noise_eta = 0.0;        // noisy kind: noise magnitude relative to ||v||
  unsigned long long seed = 0;   // noisy kind: generator key
  long long draws = 0;           // noisy kind: standalone applications so far
  // private buffers for pfk_precond_apply
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
};

// Stencil geometry for tile width tx (64: 64 x 8 tiles, 32: 32 x 16) and a
// target of about `target` workgroups (the z-range is cut into chunks).
static StencilGeom make_geom(int dim, int nx, int ny, int nz, int tx = 64, int target = 2048) {
  StencilGeom sg;
  sg.tx = tx;
  const int ty = 2 * kBlock / tx;
  sg.tiles_x = (nx + tx - 1) / tx;
  sg.tiles_y = (ny + ty - 1) / ty;
  const int tiles = sg.tiles_x * sg.tiles_y;
  int chunks = dim == 3 ? std::max(1, std::min(nz, (target + tiles - 1) / tiles)) : 1;
  sg.zc = (nz + chunks - 1) / chunks;
  sg.zchunks = (nz + sg.zc - 1) / sg.zc;
  return sg;
}

static int pointwise_blocks(long long N) {
  long long b = (N + kBlock - 1) / kBlock;
  return (int)std::max<long long>(1, std::min<long long>(b, 2048));
}

extern "C" void pfk_default_opts(pfk_solve_opts* o) {
  if (!o) return;
  o->truncation = 0;
  o->shift_sigma = NAN;
  o->graph_iters = 8;
  o->use_graph = 1;
  o->host_sync = 0;
  o->max_restarts = 10;
  o->force_breakdown_at = -1;
  o->persistent = 0;
  o->norm = 0;
  o->timestamps = 0;
  o->side_delay = 0;
  o->stall_window = 0;
}

extern "C" int pfk_operator_create(int dim, const int64_t n[3], const double* eta, const double* face_vel,
                                   int ptr_is_device, pfk_operator* out) {
  if (!out) return fail(PFK_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(PFK_ERR_ARG, "dim must be 2 or 3");
  if (!n || !eta) return fail(PFK_ERR_ARG, "n and eta are required");
  for (int a = 0; a < dim; ++a)
    if (n[a] < 1 || n[a] > 4096) return fail(PFK_ERR_ARG, "n out of range 1..4096");
  for (int a = 1; a < dim; ++a)
    if (n[a] != n[0]) return fail(PFK_ERR_ARG, "the grid must have the same n on every axis");
  if (face_vel && dim != 3) return fail(PFK_ERR_ARG, "face velocities are 3D only");
  auto* A = new (std::nothrow) pfk_operator_s();
  if (!A) return fail(PFK_ERR_OOM, "host allocation");
  A->dim = dim;
  A->n[0] = n[0];
  A->n[1] = n[1];
  A->n[2] = dim == 3 ? n[2] : 1;
  A->N = A->n[0] * A->n[1] * A->n[2];
  A->h = 1.0 / (double)(n[0] + 1);
  A->npad = (n[0] + 2) * (n[1] + 2) * (dim == 3 ? (n[2] + 2) : 1);
  A->sg = make_geom(dim, (int)A->n[0], (int)A->n[1], (int)A->n[2]);
  A->pv_blocks = pointwise_blocks(A->N);
  const hipMemcpyKind kind = ptr_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  // validate eta > 0 (host copy when given device memory)
  std::vector<double> heta((size_t)A->npad);
  if (hipMemcpy(heta.data(), eta, sizeof(double) * A->npad,
                ptr_is_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost) != hipSuccess) {
    delete A;
    return fail(PFK_ERR_HIP, "copying eta");
  }
  for (double v : heta)
    if (!(v > 0.0) || !std::isfinite(v)) {
      delete A;
      return fail(PFK_ERR_ARG, "eta must be finite and positive");
    }
  if (hipMalloc(&A->eta, sizeof(double) * A->npad) != hipSuccess ||
      hipMalloc(&A->dinv, sizeof(double) * A->N) != hipSuccess ||
      (face_vel && hipMalloc(&A->vel, 3 * sizeof(double) * A->npad) != hipSuccess)) {
    pfk_operator_destroy(A);
    return fail(PFK_ERR_OOM, "device allocation for the operator");
  }
  if (hipMemcpy(A->eta, eta, sizeof(double) * A->npad, kind) != hipSuccess ||
      (face_vel && hipMemcpy(A->vel, face_vel, 3 * sizeof(double) * A->npad, kind) != hipSuccess)) {
    pfk_operator_destroy(A);
    return fail(PFK_ERR_HIP, "copying coefficients");
  }
  hipLaunchKernelGGL(k_dinv, dim3(A->sg.blocks()), dim3(kBlock), 0, 0, A->grid(), A->sg, A->dinv);
  if (hipDeviceSynchronize() != hipSuccess) {
    pfk_operator_destroy(A);
    return fail(PFK_ERR_HIP, "computing the diagonal");
  }
  *out = A;
  return PFK_OK;
}

extern "C" void pfk_operator_destroy(pfk_operator A) {
  if (!A) return;
  if (A->eta) (void)hipFree(A->eta);
  if (A->vel) (void)hipFree(A->vel);
  if (A->dinv) (void)hipFree(A->dinv);
  if (A->eta_bf16) (void)hipFree(A->eta_bf16);
  if (A->vel_f32) (void)hipFree(A->vel_f32);
  if (A->dinv_f32) (void)hipFree(A->dinv_f32);
  delete A;
}

extern "C" int64_t pfk_operator_size(pfk_operator A) { return A ? A->N : 0; }

extern "C" int pfk_operator_apply(pfk_operator A, const double* x, double* y, void* stream) {
  if (!A || !x || !y) return fail(PFK_ERR_ARG, "null argument");
  hipLaunchKernelGGL(k_apply, dim3(A->sg.blocks()), dim3(kBlock), 0, (hipStream_t)stream, A->grid(), A->sg,
                     x, y, (const SolveState*)nullptr);
  HIPCHK(hipGetLastError());
  return PFK_OK;
}

extern "C" int pfk_operator_diag_inv(pfk_operator A, double* dinv, void* stream) {
  if (!A || !dinv) return fail(PFK_ERR_ARG, "null argument");
  HIPCHK(hipMemcpyAsync(dinv, A->dinv, sizeof(double) * A->N, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PFK_OK;
}

// Round a finite double to the nearest BF16, ties to even, directly from the
// 52-bit mantissa (no intermediate FP32 rounding).  Values here are positive
// normal numbers (viscosities).
static uint16_t bf16_rne(double x) {
  uint64_t b;
  std::memcpy(&b, &x, 8);
  const uint64_t sign = b >> 63;
  int e = (int)((b >> 52) & 0x7FF) - 1023 + 127;
  uint64_t m = b & ((1ULL << 52) - 1);
  if (x == 0.0) return (uint16_t)(sign << 15);
  uint64_t m7 = m >> 45;
  const uint64_t rem = m & ((1ULL << 45) - 1);
  const uint64_t half = 1ULL << 44;
  if (rem > half || (rem == half && (m7 & 1))) {
    ++m7;
    if (m7 == 128) { m7 = 0; ++e; }
  }
  if (e <= 0) e = 0, m7 = 0;            // flush (not reached for viscosities)
  if (e >= 255) e = 254, m7 = 127;      // clamp (not reached for viscosities)
  return (uint16_t)((sign << 15) | ((uint64_t)e << 7) | m7);
}

// BF16 eta, FP32 velocities and the FP32 D^-1 of that inner operator.
static int ensure_mixed(pfk_operator_s* A) {
  if (A->eta_bf16) return PFK_OK;
  std::vector<double> heta((size_t)A->npad);
  if (hipMemcpy(heta.data(), A->eta, sizeof(double) * A->npad, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(PFK_ERR_HIP, "reading eta");
  std::vector<uint16_t> hb((size_t)A->npad);
  for (size_t i = 0; i < hb.size(); ++i) hb[i] = bf16_rne(heta[i]);
  if (hipMalloc(&A->eta_bf16, 2 * A->npad) != hipSuccess || hipMalloc(&A->dinv_f32, 4 * A->N) != hipSuccess)
    return fail(PFK_ERR_OOM, "mixed-precision operator");
  if (hipMemcpy(A->eta_bf16, hb.data(), 2 * A->npad, hipMemcpyHostToDevice) != hipSuccess)
    return fail(PFK_ERR_HIP, "copying eta");
  if (A->vel) {
    std::vector<double> hv((size_t)(3 * A->npad));
    std::vector<float> hf(hv.size());
    if (hipMemcpy(hv.data(), A->vel, sizeof(double) * hv.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(PFK_ERR_HIP, "reading velocities");
    for (size_t i = 0; i < hv.size(); ++i) hf[i] = (float)hv[i];
    if (hipMalloc(&A->vel_f32, sizeof(float) * hf.size()) != hipSuccess) return fail(PFK_ERR_OOM, "velocities");
    if (hipMemcpy(A->vel_f32, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(PFK_ERR_HIP, "copying velocities");
  }
  hipLaunchKernelGGL(k_dinv_mixed, dim3(A->sg.blocks()), dim3(kBlock), 0, 0, A->grid_mixed(), A->sg, A->dinv_f32);
  if (hipDeviceSynchronize() != hipSuccess) return fail(PFK_ERR_HIP, "mixed diagonal");
  return PFK_OK;
}

extern "C" int pfk_precond_create(pfk_operator A, pfk_pc_kind kind, int inner_its, pfk_precision prec,
                                  int block, pfk_precond* out) {
  if (!out || !A) return fail(PFK_ERR_ARG, "null argument");
  *out = nullptr;
  if (kind == PFK_PC_NOISY) return fail(PFK_ERR_ARG, "the noisy preconditioner is made by pfk_precond_create_noisy");
  if (kind < PFK_PC_NONE || kind > PFK_PC_BLOCK_JACOBI_PCG) return fail(PFK_ERR_ARG, "unknown preconditioner");
  if ((kind == PFK_PC_JACOBI_PCG || kind == PFK_PC_JACOBI_GMRES || kind == PFK_PC_BLOCK_JACOBI_PCG) &&
      (inner_its < 1 || inner_its > kMaxInner))
    return fail(PFK_ERR_ARG, "inner_its must be 1..32");
  if (prec != PFK_FP64 && prec != PFK_FP32_BF16COEF) return fail(PFK_ERR_ARG, "unknown precision");
  if (kind == PFK_PC_JACOBI_GMRES && inner_its > kMaxInnerGmres)
    return fail(PFK_ERR_ARG, "inner GMRES supports at most 8 steps");
  if (kind == PFK_PC_BLOCK_JACOBI_PCG && block != kBjEdge)
    return fail(PFK_ERR_ARG, "block-Jacobi PCG supports blocks of 8 nodes per axis");
  if (prec == PFK_FP32_BF16COEF &&
      (kind == PFK_PC_JACOBI_PCG || kind == PFK_PC_JACOBI_GMRES || kind == PFK_PC_BLOCK_JACOBI_PCG)) {
    const int rc = ensure_mixed(A);
    if (rc) return rc;
  }
  auto* B = new (std::nothrow) pfk_precond_s();
  if (!B) return fail(PFK_ERR_OOM, "host allocation");
  B->A = A;
  B->kind = kind;
  B->k = (kind == PFK_PC_NONE || kind == PFK_PC_JACOBI) ? 1 : inner_its;
  B->prec = prec;
  B->block = block;
  *out = B;
  return PFK_OK;
}

extern "C" int pfk_precond_create_noisy(pfk_operator A, double eta, uint64_t seed, pfk_precond* out) {
  if (!out || !A) return fail(PFK_ERR_ARG, "null argument");
  *out = nullptr;
  if (!(eta >= 0.0) || !std::isfinite(eta)) return fail(PFK_ERR_ARG, "eta must be finite and non-negative");
  auto* B = new (std::nothrow) pfk_precond_s();
  if (!B) return fail(PFK_ERR_OOM, "host allocation");
  B->A = A;
  B->kind = PFK_PC_NOISY;
  B->k = 1;
  B->prec = PFK_FP64;
  B->noise_eta = eta;
  B->seed = (unsigned long long)seed;
  *out = B;
  return PFK_OK;
}

extern "C" void pfk_precond_destroy(pfk_precond B) {
  if (!B) return;
  if (B->scratch) (void)hipFree(B->scratch);
  delete B;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

enum Vec {
  V_R, V_U, V_W, V_M, V_N,                       // outer work vectors
  V_PC_Q, V_PC_RHO, V_PC_Y,                      // inner PCG (its directions: window W_PCP)
  V_X0, V_Z, V_VIN,                              // GMRES family: cycle start x, z / wbar, basis input
  V_COUNT
};
enum Win { W_P, W_S, W_Q, W_Z, W_PCV, W_PCP, W_COUNT };  // W_PCV: inner GMRES basis; W_PCP: inner PCG directions
enum Part { PT_MAIN, PT_A, PT_B, PT_PC0, PT_PC1, PT_COUNT };

struct Layout {
  size_t state = 0, hist = 0, nhist = 0, tstamp = 0;
  size_t vec[V_COUNT] = {};
  size_t win[W_COUNT] = {};
  int slots[W_COUNT] = {};
  size_t part[PT_COUNT] = {};
  long long ld = 0;
  size_t total = 0;
};

// Window slots per method: CG/CR types keep nu_max directions in P, S (and
// Q, Z for the pipelined ones); GMRES types keep the basis P (m+1 columns),
// U (m, or m+1 for PIPEFGMRES) and PIPEFGMRES's zbar (m+1).
void window_slots(int method, int mmax, int* slots) {
  for (int w = 0; w < W_COUNT; ++w) slots[w] = 0;
  switch (method) {
    case PFK_FCG: case PFK_GCR: slots[W_P] = slots[W_S] = mmax; break;
    case PFK_PIPEGCR: slots[W_P] = slots[W_S] = slots[W_Q] = mmax; break;
    case PFK_PIPEFCG: case PFK_PIPEGCR_W: case PFK_PIPEFCG_NAIVE:
      slots[W_P] = slots[W_S] = slots[W_Q] = slots[W_Z] = mmax;
      break;
    case PFK_FGMRES: slots[W_P] = mmax + 1; slots[W_S] = mmax; break;
    case PFK_PIPEFGMRES: slots[W_P] = slots[W_S] = slots[W_Q] = mmax + 1; break;
    default: break;
  }
}

// pmin: partial-sum arrays hold at least pmin workgroups (the autotuner's
// largest candidate); otherwise the operator's current launch geometry.
Layout make_layout(const pfk_operator_s* A, const pfk_precond_s* B, int method, int mmax, int maxit,
                   int pmin = 0) {
  Layout L;
  size_t off = 0;
  L.state = off;
  off = align_up(off + sizeof(SolveState));
  L.hist = off;
  off = align_up(off + sizeof(double) * (size_t)(maxit + 2));
  L.nhist = off;
  off = align_up(off + sizeof(double) * (size_t)(maxit + 2));
  L.tstamp = off;
  off = align_up(off + sizeof(unsigned long long) * (size_t)(maxit + 2));
  L.ld = (A->N + 31) / 32 * 32;
  const size_t vbytes = align_up(sizeof(double) * (size_t)L.ld);
  for (int v = 0; v < V_COUNT; ++v) {
    L.vec[v] = off;
    off += vbytes;
  }
  window_slots(method, mmax, L.slots);
  if (B && B->kind == PFK_PC_JACOBI_GMRES) L.slots[W_PCV] = B->k + 1;
  if (B && B->kind == PFK_PC_JACOBI_PCG) L.slots[W_PCP] = B->k;
  for (int w = 0; w < W_COUNT; ++w) {
    L.win[w] = off;
    off += vbytes * (size_t)L.slots[w];
  }
  const int P = std::max(std::max(A->sg.blocks(), A->pv_blocks), pmin);
  const size_t pbytes = align_up(sizeof(double) * (size_t)P * (kNuMax + 4));
  for (int p = 0; p < PT_COUNT; ++p) {
    L.part[p] = off;
    off += pbytes;
  }
  L.total = off;
  return L;
}

}  // namespace

extern "C" size_t pfk_workspace_bytes(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int maxit) {
  if (!A || mmax < 1 || mmax > kNuMax || maxit < 0) return 0;
  return make_layout(A, B, method, mmax, maxit).total;
}

// ---------------------------------------------------------------------------
// sessions
// ---------------------------------------------------------------------------
// Unknowns (times the batch capacity for batch members) from which the
// vector kernels stream with nontemporal accesses: below it the L2 and the
// Infinity Cache keep a solve's vectors between kernels.
constexpr double kNtMinUnknowns = 1 << 20;

struct pfk_session_s {
  pfk_operator A = nullptr;
  pfk_precond B = nullptr;
  int method = 0;
  const double* b = nullptr;
  double* x = nullptr;
  double rtol = 0.0;
  int maxit = 0, mmax = 0;
  double sigma = 0.0;
  pfk_solve_opts opts{};
  int nt_scale = 1;                 // batch members: the batch capacity
  char* ws = nullptr;
  bool ws_owned = false;
  Layout L;
  hipStream_t user = nullptr, s1 = nullptr, s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_user = nullptr, ev_done = nullptr;
  hipGraphExec_t g_start = nullptr, g_iter = nullptr, g_one = nullptr;
  SolveState* st = nullptr;
  double* hist = nullptr;
  double* nhist = nullptr;
  unsigned long long* tstamp = nullptr;
  SolveState* host_state = nullptr;   // pinned
  int restarts = 0;
  bool owns_streams = true;           // false for members of a batch (the batch's streams)

  double* vec(int v) const { return (double*)(ws + L.vec[v]); }
  Window win(int w) const { return Window{(double*)(ws + L.win[w]), L.ld}; }
  double* part(int p) const { return (double*)(ws + L.part[p]); }
  Grid grid() const { return A->grid(); }
  // launch geometry, fixed when the session is made (the workspace's
  // partial-sum arrays are sized for it)
  StencilGeom sg{};
  int pv = 0;
  int Ps() const { return sg.blocks(); }
  int Pv() const { return pv; }
  long long noise_draw = -1;          // noisy PC: fixed draw index (standalone apply), or -1
  int noise_apps = 0;                 // noisy PC: applications enqueued in the current phase
};

// Nontemporal vector accesses once the solve's working set (the members of a
// batch together) is far beyond the caches.
inline int session_nt(const pfk_session_s* S) {
  return (double)S->A->N * S->nt_scale >= kNtMinUnknowns ? 1 : 0;
}

namespace {

// Optional per-kernel timing (pfk_session_profile): HIP events recorded on
// the launching stream immediately before and after each kernel.
struct KernelProfiler {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~KernelProfiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
thread_local KernelProfiler* g_prof = nullptr;

#define LAUNCH(kernel, blocks, stream, ...)                                              \
  do {                                                                                   \
    hipEvent_t ea_ = nullptr;                                                            \
    if (g_prof) {                                                                        \
      ea_ = g_prof->get();                                                               \
      (void)hipEventRecord(ea_, stream);                                                 \
    }                                                                                    \
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlock), 0, stream, __VA_ARGS__);      \
    if (g_prof) {                                                                        \
      hipEvent_t eb_ = g_prof->get();                                                    \
      (void)hipEventRecord(eb_, stream);                                                 \
      g_prof->recs.push_back({#kernel, ea_, eb_});                                       \
    }                                                                                    \
  } while (0)

// A stencil kernel in its convective form (kernel_cv) when the operator has
// face velocities.
#define LAUNCH_OP(op, kernel, blocks, stream, ...)                                       \
  do {                                                                                   \
    if ((op)->vel != nullptr) LAUNCH(kernel##_cv, blocks, stream, __VA_ARGS__);          \
    else LAUNCH(kernel, blocks, stream, __VA_ARGS__);                                    \
  } while (0)

// k_apply_pc_out in the instantiation for the descriptor's output kind.
#define LAUNCH_PC_OUT(pd, blocks, stream, ...)                                                      \
  do {                                                                                              \
    if ((pd).kind == kPcBlockPcg) {                                                                 \
      if ((pd).fp32) LAUNCH((k_apply_pc_out<kPcBlockPcg, 1>), blocks, stream, __VA_ARGS__);         \
      else LAUNCH((k_apply_pc_out<kPcBlockPcg, 0>), blocks, stream, __VA_ARGS__);                   \
    } else if ((pd).kind == kPcJacobiPcg) {                                                         \
      if ((pd).fp32) LAUNCH((k_apply_pc_out<kPcJacobiPcg, 1>), blocks, stream, __VA_ARGS__);        \
      else LAUNCH((k_apply_pc_out<kPcJacobiPcg, 0>), blocks, stream, __VA_ARGS__);                  \
    } else if ((pd).kind == kPcJacobiGmres && (pd).fp32 && (pd).k <= kGmRaw) {                      \
      LAUNCH((k_apply_pc_out<kPcJacobiGmres, 1>), blocks, stream, __VA_ARGS__);                     \
    } else {                                                                                        \
      LAUNCH((k_apply_pc_out<-1, 0>), blocks, stream, __VA_ARGS__);                                 \
    }                                                                                               \
  } while (0)

// Enqueue the inner solve B(v), v = c1*X1 + c2*X2; returns how the consumer
// evaluates B(v).
// How a consumer evaluates B(v) after enqueue_pc(v): which buffers hold the
// inner solve's last state (the same buffers every time).
PcOutDesc pc_out_desc(const pfk_session_s* S, const double* X1, double c1, const double* X2, double c2) {
  PcOutDesc d{};
  d.kind = S->B->kind;
  d.k = S->B->k;
  if (d.kind == PFK_PC_NOISY) {
    // the noisy output is stored whole; consumers read it as block PCG's
    d.kind = kPcBlockPcg;
    d.fp32 = 0;
    d.X1 = X1; d.c1 = c1; d.X2 = X2; d.c2 = c2;
    d.dinv = S->A->dinv;
    d.dinv_in = S->A->dinv;
    d.y = S->vec(V_PC_Y);
    return d;
  }
  d.fp32 = S->B->prec == PFK_FP32_BF16COEF &&
           (d.kind == kPcJacobiPcg || d.kind == kPcJacobiGmres || d.kind == kPcBlockPcg);
  d.X1 = X1; d.c1 = c1; d.X2 = X2; d.c2 = c2;
  d.dinv = S->A->dinv;
  d.dinv_in = d.fp32 ? (const void*)S->A->dinv_f32 : (const void*)S->A->dinv;
  if (d.kind == kPcJacobiPcg) {
    // A_1, (B_j, A_{j+1}) alternate the partial buffers: A_k writes PC0
    d.y = S->vec(V_PC_Y);
    d.pk = (const char*)S->win(W_PCP).base +
           (size_t)(d.k - 1) * (size_t)S->L.ld * (d.fp32 ? sizeof(float) : sizeof(double));
    d.part = S->part(PT_PC0);
    d.P = S->Ps();
  } else if (d.kind == kPcBlockPcg) {
    d.y = S->vec(V_PC_Y);
  } else if (d.kind == kPcJacobiGmres) {
    // the inner solve's end (k_gmpc_finish) leaves the coefficients in the
    // solve's scalars
    d.vbase = S->win(W_PCV).base;
    d.ldv = S->L.ld;
  }
  return d;
}

// GF_j of the inner GMRES: one instantiation per basis length up to
// kGfFixed (their raw loads fixed at compile time), one for longer bases.
template <class T, class G, bool CV>
void launch_gmpc_fused_cv(pfk_session_s* S, hipStream_t s, int j, int k, const G& g, const T* dinv,
                          const double* X1, double c1, const double* X2, double c2, T* V, long long ldv,
                          const T* wp, T* wo, const double* pin, int Pin, double* pout) {
#define PFK_GF(J)                                                                                            \
  do {                                                                                                       \
    if (j + 1 == k)                                                                                          \
      LAUNCH((k_gmpc_fused<T, G, CV, J, true>), S->Ps(), s, j, k, g, S->sg, dinv, X1, c1, X2, c2, V, ldv, wp,  \
             wo, pin, Pin, pout, S->st);                                                                     \
    else                                                                                                     \
      LAUNCH((k_gmpc_fused<T, G, CV, J, false>), S->Ps(), s, j, k, g, S->sg, dinv, X1, c1, X2, c2, V, ldv, wp, \
             wo, pin, Pin, pout, S->st);                                                                     \
  } while (0)
  switch (j) {
    case 0: PFK_GF(0); break;
    case 1: PFK_GF(1); break;
    case 2: PFK_GF(2); break;
    case 3: PFK_GF(3); break;
    case 4: PFK_GF(4); break;
    default: PFK_GF(kGfFixed + 1); break;
  }
#undef PFK_GF
}
template <class T, class G>
void launch_gmpc_fused(pfk_session_s* S, hipStream_t s, bool cv, int j, int k, const G& g, const T* dinv,
                       const double* X1, double c1, const double* X2, double c2, T* V, long long ldv,
                       const T* wp, T* wo, const double* pin, int Pin, double* pout) {
  if (cv) launch_gmpc_fused_cv<T, G, true>(S, s, j, k, g, dinv, X1, c1, X2, c2, V, ldv, wp, wo, pin, Pin, pout);
  else launch_gmpc_fused_cv<T, G, false>(S, s, j, k, g, dinv, X1, c1, X2, c2, V, ldv, wp, wo, pin, Pin, pout);
}

// The inner solve's kernels in arithmetic type T on operator description G
// (FP64 on the outer operator, or FP32 on the BF16 one).  Its work vectors
// are the session's inner vectors viewed as T.
template <class T, class G>
void enqueue_pc_kernels(pfk_session_s* S, hipStream_t s, const PcOutDesc& d, const G& g, const T* dinv) {
  const pfk_operator_s* A = S->A;
  const double *X1 = d.X1, *X2 = d.X2;
  const double c1 = d.c1, c2 = d.c2;
  double* part[2] = {S->part(PT_PC0), S->part(PT_PC1)};
  if (d.kind == kPcJacobiPcg) {
    // directions p_1 .. p_k in the window's slots 0 .. k-1 (T elements, ld apart)
    T* Pb = (T*)S->win(W_PCP).base;
    const long long ldp = S->L.ld;
    T* q = (T*)S->vec(V_PC_Q);
    T* rho = (T*)S->vec(V_PC_RHO);
    T* y = (T*)S->vec(V_PC_Y);
    LAUNCH((k_pcg_a1<T, G>), S->Ps(), s, g, S->sg, dinv, X1, c1, X2, c2, Pb, q, part[0],
           (const SolveState*)S->st);
    int t = 1, Pprev = S->Ps();
    for (int j = 1; j < d.k; ++j) {
      LAUNCH((k_pcg_b<T>), S->Pv(), s, j, d.k, A->N, dinv, X1, c1, X2, c2, (const T*)Pb, ldp, (const T*)q, rho,
             y, (const double*)part[(t - 1) & 1], Pprev, part[t & 1], S->st);
      Pprev = S->Pv();
      ++t;
      LAUNCH((k_pcg_a<T, G>), S->Ps(), s, j + 1, g, S->sg, dinv, (const T*)rho, (const T*)(Pb + (j - 1) * ldp),
             Pb + j * ldp, q, (const double*)part[(t - 1) & 1], Pprev, part[t & 1], S->st);
      Pprev = S->Ps();
      ++t;
    }
  } else if (d.kind == kPcBlockPcg) {
    T* y = (T*)S->vec(V_PC_Y);
    const int wy = ((int)A->n[1] + kBjEdge - 1) / kBjEdge;
    if (A->dim == 3) {
      const int wx = (int)((A->n[0] + 2 * kBjEdge - 1) / (2 * kBjEdge));
      const int wz = (int)((A->n[2] + kBjEdge - 1) / kBjEdge);
      LAUNCH((k_block_pcg<T, G, 1>), wx * wy * wz, s, g, wx, wy, d.k, X1, c1, X2, c2, y, (const SolveState*)S->st);
    } else {
      const int wx = (int)((A->n[0] + 4 * kBjEdge - 1) / (4 * kBjEdge));
      LAUNCH((k_block_pcg<T, G, 0>), wx * wy, s, g, wx, wy, d.k, X1, c1, X2, c2, y, (const SolveState*)S->st);
    }
  } else if (d.kind == kPcJacobiGmres) {
    T* V = (T*)S->win(W_PCV).base;
    const long long ldv = S->L.ld;
    // w~ alternates between the inner vector and the basis window's last slot
    T* w[2] = {(T*)S->vec(V_PC_Q), V + (long long)d.k * ldv};
    const bool cv = A->vel != nullptr;
    for (int j = 0; j < d.k; ++j) {
      // GF_j reads GF_{j-1}'s partials and writes its own (PC0 and PC1 in turn)
      const T* wp = j > 0 ? (const T*)w[(j - 1) & 1] : nullptr;
      launch_gmpc_fused<T, G>(S, s, cv, j, d.k, g, dinv, X1, c1, X2, c2, V, ldv, wp, w[j & 1],
                              (const double*)part[(j + 1) & 1], S->Ps(), part[j & 1]);
    }
    LAUNCH(k_gmpc_finish, 1, s, d.k, (const double*)part[(d.k - 1) & 1], S->Ps(), S->st);
  }
}

// Enqueue the inner solve B(v), v = c1*X1 + c2*X2; returns how the consumer
// evaluates B(v).
PcOutDesc enqueue_pc(pfk_session_s* S, hipStream_t s, const double* X1, double c1, const double* X2,
                     double c2) {
  const PcOutDesc d = pc_out_desc(S, X1, c1, X2, c2);
  if (S->B->kind == PFK_PC_NOISY) {
    const long long N = S->A->N;
    const int off = S->noise_apps++;
    LAUNCH(k_noise_norms, S->Pv(), s, N, X1, c1, X2, c2, S->B->seed, S->noise_draw, off, S->part(PT_PC0),
           (const SolveState*)S->st);
    LAUNCH(k_noise_apply, S->Pv(), s, N, X1, c1, X2, c2, S->B->seed, S->noise_draw, off, S->B->noise_eta,
           (const double*)S->part(PT_PC0), S->Pv(), S->vec(V_PC_Y), (const SolveState*)S->st);
    return d;
  }
  if (d.fp32) enqueue_pc_kernels<float>(S, s, d, S->A->grid_mixed(), (const float*)S->A->dinv_f32);
  else enqueue_pc_kernels<double>(S, s, d, S->grid(), (const double*)S->A->dinv);
  return d;
}

// Phase bracket of the noisy preconditioner's draw count (no-ops otherwise).
void noise_begin(pfk_session_s* S, hipStream_t s) {
  S->noise_apps = 0;
  if (S->B->kind == PFK_PC_NOISY) LAUNCH(k_noise_mark, 1, s, S->st);
}
void noise_end(pfk_session_s* S, hipStream_t s) {
  if (S->B->kind == PFK_PC_NOISY && S->noise_apps > 0) LAUNCH(k_noise_advance, 1, s, S->st, S->noise_apps);
  S->noise_apps = 0;
}

void enqueue_multidot(pfk_session_s* S, hipStream_t s, int init, int from_pc, const PcOutDesc& pd,
                      const double* Vin, double* Vout) {
  LAUNCH(k_multidot, S->Pv(), s, S->A->N, init, from_pc, pd, Vin, Vout, (const double*)S->vec(V_R),
         S->win(W_S), S->part(PT_MAIN), S->st);
}

// The host-sync form of the unpipelined baselines: a reduction's result is
// copied to the host, which waits for it before enqueuing more work (the
// analogue of a blocking all-reduce).  host_sync turns graphs off, so this
// never runs under capture.
void host_wait(pfk_session_s* S, hipStream_t s) {
  if (!S->opts.host_sync) return;
  (void)hipMemcpyAsync(&S->host_state->gamma, &S->st->gamma, sizeof(double), hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
}

// FCG / GCR: the part of an iteration after x, r have been updated, also
// the start-up (init = 1).
//   FCG: u = B(r); reduction 1 (<u,r>, <r,r>, <u,s_d>); p = u + sum beta p;
//        s = A p with reduction 2 (<p,s>)
//   GCR: u = B(r), t = A u; reduction 1 (<r,r>, <t,s_d>); p = u + sum beta p,
//        s = t + sum beta s with reduction 2 (<r,s>, <s,s>)
void enqueue_cg_body(pfk_session_s* S, hipStream_t s, int init) {
  const Grid g = S->grid();
  PcOutDesc pd = enqueue_pc(S, s, S->vec(V_R), 1.0, nullptr, 0.0);
  if (S->method == PFK_FCG) {
    enqueue_multidot(S, s, init, 1, pd, nullptr, S->vec(V_U));
    LAUNCH(k_cg_scalars1, 1, s, init, S->part(PT_MAIN), S->Pv(), S->st, S->hist);
    host_wait(S, s);
    LAUNCH(k_fcg_maxpy, S->Pv(), s, S->A->N, S->win(W_P), (const double*)S->vec(V_U), (const SolveState*)S->st);
    LAUNCH(k_fcg_apply, S->Ps(), s, g, S->sg, S->win(W_P), S->win(W_S), S->part(PT_A), (const SolveState*)S->st);
    LAUNCH(k_cg_scalars2, 1, s, 0, init, S->part(PT_A), S->Ps(), S->st);
    host_wait(S, s);
  } else {
    LAUNCH_PC_OUT(pd, S->Ps(), s, g, S->sg, pd, (const double*)nullptr, 0.0, S->vec(V_U), S->vec(V_W), 0,
           (const double*)nullptr, S->part(PT_B), S->st);
    enqueue_multidot(S, s, init, 0, pd, S->vec(V_W), nullptr);
    LAUNCH(k_cg_scalars1, 1, s, init, S->part(PT_MAIN), S->Pv(), S->st, S->hist);
    host_wait(S, s);
    LAUNCH(k_gcr_maxpy, S->Pv(), s, S->A->N, S->win(W_P), S->win(W_S), (const double*)S->vec(V_U),
           (const double*)S->vec(V_W), (const double*)S->vec(V_R), S->part(PT_A), (const SolveState*)S->st);
    LAUNCH(k_cg_scalars2, 1, s, 1, init, S->part(PT_A), S->Pv(), S->st);
    host_wait(S, s);
  }
}

// Start (or restart) from the current x.
void enqueue_start(pfk_session_s* S, hipStream_t s) {
  const pfk_operator_s* A = S->A;
  const Grid g = S->grid();
  const bool gm = S->method == PFK_FGMRES || S->method == PFK_PIPEFGMRES;
  LAUNCH(k_restart, 1, s, S->st);
  noise_begin(S, s);
  LAUNCH(k_residual, S->Ps(), s, g, S->sg, S->b, (const double*)S->x, S->vec(V_R), S->part(PT_A),
         gm ? S->vec(V_X0) : nullptr);
  switch (S->method) {
    case PFK_FCG:
    case PFK_GCR:
      LAUNCH(k_init_test, 1, s, S->part(PT_A), S->Ps(), S->st, S->hist);
      enqueue_cg_body(S, s, 1);
      break;
    case PFK_PIPEFCG:
    case PFK_PIPEFCG_NAIVE:
    case PFK_PIPEGCR_W: {
      // u_0 = B(r_0), w_0 = A u_0; PIPEFCG: gamma_0 = <u_0,r_0>, eta_0 = <u_0,w_0>;
      // PIPEGCR_w (p_0 = u_0, s_0 = w_0): gamma_0 = <r_0,s_0>, eta_0 = <s_0,s_0>
      const int dots = S->method == PFK_PIPEGCR_W ? 2 : 1;
      PcOutDesc pd = enqueue_pc(S, s, S->vec(V_R), 1.0, nullptr, 0.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s, g, S->sg, pd, (const double*)nullptr, 0.0, S->vec(V_U), S->vec(V_W), dots,
             (const double*)S->vec(V_R), S->part(PT_B), S->st);
      // m_0 = B(w_0), n_0 = A m_0
      pd = enqueue_pc(S, s, S->vec(V_W), 1.0, nullptr, 0.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s, g, S->sg, pd, (const double*)nullptr, 0.0, S->vec(V_M), S->vec(V_N), 0,
             (const double*)nullptr, S->part(PT_B), S->st);
      LAUNCH(k_pipefcg_init_scalars, 1, s, S->part(PT_A), S->Ps(), S->part(PT_B), S->Ps(), S->st, S->hist);
      break;
    }
    case PFK_PIPEGCR: {
      LAUNCH(k_init_test, 1, s, S->part(PT_A), S->Ps(), S->st, S->hist);
      // u_0 = B(r_0), s_0 = A u_0 (kept in w), gamma_0 = <r_0,s_0>, eta_0 = <s_0,s_0>
      PcOutDesc pd = enqueue_pc(S, s, S->vec(V_R), 1.0, nullptr, 0.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s, g, S->sg, pd, (const double*)nullptr, 0.0, S->vec(V_U), S->vec(V_W), 0,
             (const double*)nullptr, S->part(PT_B), S->st);
      enqueue_multidot(S, s, 1, 0, pd, S->vec(V_W), nullptr);
      // q_0 = B(s_0), consumed by the first update
      enqueue_pc(S, s, S->vec(V_W), 1.0, nullptr, 0.0);
      LAUNCH(k_pipegcr_init_scalars, 1, s, S->part(PT_MAIN), S->Pv(), S->st);
      break;
    }
    case PFK_FGMRES:
      LAUNCH(k_gm_cycle_start, 1, s, S->part(PT_A), S->Ps(), S->st, S->hist);
      LAUNCH(k_gm_scale, S->Pv(), s, A->N, (const double*)S->vec(V_R), 0, S->win(W_P), S->vec(V_VIN),
             (const SolveState*)S->st);
      break;
    case PFK_PIPEFGMRES: {
      LAUNCH(k_gm_cycle_start, 1, s, S->part(PT_A), S->Ps(), S->st, S->hist);
      LAUNCH(k_gm_scale, S->Pv(), s, A->N, (const double*)S->vec(V_R), 0, S->win(W_P), S->vec(V_VIN),
             (const SolveState*)S->st);
      // u~_0 = B(p_0), zbar_0 = A u~_0 - sigma p_0, first reduction
      PcOutDesc pd = enqueue_pc(S, s, S->vec(V_VIN), 1.0, nullptr, 0.0);
      LAUNCH(k_pgm_apply0, S->Ps(), s, g, S->sg, pd, S->win(W_S), S->win(W_P), S->win(W_Q), S->vec(V_M),
             S->part(PT_MAIN), S->st);
      // qbar_0 = B(zbar_0), wbar_0 = A qbar_0
      pd = enqueue_pc(S, s, S->vec(V_M), 1.0, nullptr, 0.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s, g, S->sg, pd, (const double*)nullptr, 0.0, (double*)nullptr,
             S->vec(V_Z), 0, (const double*)nullptr, S->part(PT_B), S->st);
      LAUNCH(k_pgm_scalars, 1, s, S->part(PT_MAIN), S->Ps(), S->st, S->hist);   // partials of k_pgm_apply0
      LAUNCH(k_gm_update_x, S->Pv(), s, A->N, S->win(W_S), (const double*)S->vec(V_X0), S->x,
             (const SolveState*)S->st);
      break;
    }
    default:
      break;
  }
  noise_end(S, s);
}

// The second stream's branch of a pipelined iteration: fork it off s1, mark
// its end, join it back.  A session that runs on one stream (s1 == s2) has
// no events and orders the same kernels in one queue (same results).
void side_fork(pfk_session_s* S) {
  if (S->s2 == S->s1) return;
  (void)hipEventRecord(S->ev_fork, S->s1);
  (void)hipStreamWaitEvent(S->s2, S->ev_fork, 0);
}
void side_end(pfk_session_s* S) {
  if (S->s2 != S->s1) (void)hipEventRecord(S->ev_join, S->s2);
}
void side_join(pfk_session_s* S) {
  if (S->s2 != S->s1) (void)hipStreamWaitEvent(S->s1, S->ev_join, 0);
}

// The stream-join test hook (opts.side_delay): a bounded delay on stream s.
void side_delay(const pfk_session_s* S, hipStream_t s) {
  if (S->opts.side_delay > 0) LAUNCH(k_delay, 1, s, S->opts.side_delay);
}

// One iteration.
void enqueue_iteration(pfk_session_s* S) {
  const pfk_operator_s* A = S->A;
  const Grid g = S->grid();
  hipStream_t s1 = S->s1, s2 = S->s2;
  noise_begin(S, s1);
  switch (S->method) {
    case PFK_FCG:
    case PFK_GCR:
      LAUNCH(k_fcg_xr, S->Pv(), s1, A->N, S->win(W_P), S->win(W_S), S->x, S->vec(V_R), (const SolveState*)S->st);
      enqueue_cg_body(S, s1, 0);
      break;
    case PFK_PIPEFCG:
    case PFK_PIPEFCG_NAIVE:
    case PFK_PIPEGCR_W: {
      LAUNCH(k_pipefcg_update, S->Pv(), s1, A->N, S->win(W_P), S->win(W_S), S->win(W_Q), S->win(W_Z), S->x,
             S->vec(V_R), S->vec(V_U), S->vec(V_W), (const double*)S->vec(V_M), (const double*)S->vec(V_N),
             S->part(PT_MAIN), (const SolveState*)S->st, S->method == PFK_PIPEGCR_W ? 1 : 0);
      // fork: finish the reduction on s2 while s1 applies B and A
      side_fork(S);
      side_delay(S, s2);
      LAUNCH(k_pipefcg_scalars, 1, s2, S->part(PT_MAIN), S->Pv(), S->st, S->hist);
      side_end(S);
      // m = u + B(w - r) (Alg. 8, 12); the naive form (Alg. 7) takes m = B(w)
      const bool naive = S->method == PFK_PIPEFCG_NAIVE;
      PcOutDesc pd = naive ? enqueue_pc(S, s1, S->vec(V_W), 1.0, nullptr, 0.0)
                           : enqueue_pc(S, s1, S->vec(V_W), 1.0, S->vec(V_R), -1.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s1, g, S->sg, pd, naive ? (const double*)nullptr : (const double*)S->vec(V_U),
             naive ? 0.0 : 1.0, S->vec(V_M), S->vec(V_N), 0, (const double*)nullptr, S->part(PT_B), S->st);
      side_join(S);
      break;
    }
    case PFK_PIPEGCR: {
      // the inner solve's output of the previous iteration: B(w - r)
      const PcOutDesc pd_prev = pc_out_desc(S, S->vec(V_W), 1.0, S->vec(V_R), -1.0);
      LAUNCH(k_pipegcr_update, S->Pv(), s1, A->N, S->win(W_P), S->win(W_S), S->win(W_Q), S->x, S->vec(V_R),
             S->vec(V_U), (const double*)S->vec(V_W), pd_prev, S->st);
      LAUNCH_OP(S->A, k_apply, S->Ps(), s1, g, S->sg, (const double*)S->vec(V_U), S->vec(V_W), (const SolveState*)S->st);
      enqueue_multidot(S, s1, 0, 0, pd_prev, S->vec(V_W), nullptr);
      side_fork(S);
      side_delay(S, s2);
      LAUNCH(k_pipefcg_scalars, 1, s2, S->part(PT_MAIN), S->Pv(), S->st, S->hist);
      side_end(S);
      enqueue_pc(S, s1, S->vec(V_W), 1.0, S->vec(V_R), -1.0);
      side_join(S);
      break;
    }
    case PFK_FGMRES: {
      PcOutDesc pd = enqueue_pc(S, s1, S->vec(V_VIN), 1.0, nullptr, 0.0);
      LAUNCH(k_fgm_apply, S->Ps(), s1, g, S->sg, pd, S->win(W_S), S->vec(V_Z), S->st);
      LAUNCH(k_fgm_dots, S->Pv(), s1, A->N, S->win(W_P), (const double*)S->vec(V_Z), S->part(PT_MAIN),
             (const SolveState*)S->st);
      LAUNCH(k_gm_hbar, 1, s1, S->part(PT_MAIN), S->Pv(), S->st);
      host_wait(S, s1);
      LAUNCH(k_fgm_orth, S->Pv(), s1, A->N, S->win(W_P), (const double*)S->vec(V_Z), S->part(PT_A),
             (const SolveState*)S->st);
      LAUNCH(k_fgm_column, 1, s1, S->part(PT_A), S->Pv(), S->st, S->hist);
      host_wait(S, s1);
      LAUNCH(k_gm_scale, S->Pv(), s1, A->N, (const double*)nullptr, 1, S->win(W_P), S->vec(V_VIN),
             (const SolveState*)S->st);
      LAUNCH(k_gm_update_x, S->Pv(), s1, A->N, S->win(W_S), (const double*)S->vec(V_X0), S->x,
             (const SolveState*)S->st);
      break;
    }
    case PFK_PIPEFGMRES: {
      // the inner solve's output of the previous iteration: qbar = B(zbar)
      const PcOutDesc pd_prev = pc_out_desc(S, S->vec(V_M), 1.0, nullptr, 0.0);
      LAUNCH(k_pgm_update, S->Pv(), s1, A->N, S->win(W_P), S->win(W_S), S->win(W_Q), pd_prev,
             (const double*)S->vec(V_Z), S->vec(V_M), S->part(PT_MAIN), S->st);
      side_fork(S);
      side_delay(S, s2);
      LAUNCH(k_pgm_scalars, 1, s2, S->part(PT_MAIN), S->Pv(), S->st, S->hist);
      side_end(S);
      PcOutDesc pd = enqueue_pc(S, s1, S->vec(V_M), 1.0, nullptr, 0.0);
      LAUNCH_PC_OUT(pd, S->Ps(), s1, g, S->sg, pd, (const double*)nullptr, 0.0, (double*)nullptr,
             S->vec(V_Z), 0, (const double*)nullptr, S->part(PT_B), S->st);
      side_join(S);
      LAUNCH(k_gm_update_x, S->Pv(), s1, A->N, S->win(W_S), (const double*)S->vec(V_X0), S->x,
             (const SolveState*)S->st);
      break;
    }
    default:
      break;
  }
  noise_end(S, s1);
}

// Whether the solve tests the natural norm (CG/CR types with opts.norm = 1).
bool natural_mode(const pfk_session_s* S) {
  const bool gm = S->method == PFK_FGMRES || S->method == PFK_PIPEFGMRES;
  return S->opts.norm == 1 && !gm;
}
bool cr_type(int method) { return method == PFK_GCR || method == PFK_PIPEGCR || method == PFK_PIPEGCR_W; }

// The verdict after a recurred convergence (status kConverged): r = b - A x,
// then in the 2-norm mode ||r|| <= tol, in the natural-norm mode
// sqrt|<B(r), r>| (CR types sqrt|<r, A B(r)>|) <= rtol times the natural norm
// of the first start-up -- unless the first start-up met the 2-norm
// tolerance before any natural norm existed, when the 2-norm decides.
void enqueue_true_check(pfk_session_s* S, hipStream_t s) {
  LAUNCH(k_residual, S->Ps(), s, S->grid(), S->sg, S->b, (const double*)S->x, S->vec(V_R), S->part(PT_A),
         (double*)nullptr);
  if (!natural_mode(S)) {
    LAUNCH(k_true_check, 1, s, S->part(PT_A), S->Ps(), (const double*)nullptr, 0, S->st);
    return;
  }
  const long long N = S->A->N;
  LAUNCH(k_check_open, 1, s, S->st);
  noise_begin(S, s);
  const PcOutDesc pd = enqueue_pc(S, s, S->vec(V_R), 1.0, nullptr, 0.0);
  LAUNCH(k_pc_write, S->Pv(), s, N, pd, S->vec(V_U), S->st);
  noise_end(S, s);
  if (cr_type(S->method)) {
    LAUNCH_OP(S->A, k_apply, S->Ps(), s, S->grid(), S->sg, (const double*)S->vec(V_U), S->vec(V_W),
              (const SolveState*)S->st);
    LAUNCH(k_dot, S->Pv(), s, N, (const double*)S->vec(V_R), (const double*)S->vec(V_W), S->part(PT_B));
  } else {
    LAUNCH(k_dot, S->Pv(), s, N, (const double*)S->vec(V_U), (const double*)S->vec(V_R), S->part(PT_B));
  }
  LAUNCH(k_true_check, 1, s, S->part(PT_A), S->Ps(), (const double*)S->part(PT_B), S->Pv(), S->st);
}

// ||b - A x|| at exit, for the report (status unchanged).
void enqueue_true_residual(pfk_session_s* S, hipStream_t s) {
  LAUNCH(k_residual, S->Ps(), s, S->grid(), S->sg, S->b, (const double*)S->x, S->vec(V_R), S->part(PT_A),
         (double*)nullptr);
  LAUNCH(k_true_report, 1, s, S->part(PT_A), S->Ps(), S->st);
}

// sigma of PIPEFGMRES: Rayleigh quotient of v -> A B(v) after `its` power steps
// from the normalised ones vector.  Uses the session's work vectors.
void enqueue_sigma_estimate(pfk_session_s* S, hipStream_t s, int its) {
  const pfk_operator_s* A = S->A;
  double* v = S->vec(V_VIN);
  double* w = S->vec(V_Z);
  LAUNCH(k_set_running, 1, s, S->st, session_nt(S));
  noise_begin(S, s);
  LAUNCH(k_fill, S->Pv(), s, A->N, v, 1.0 / std::sqrt((double)A->N));
  for (int i = 0; i < its; ++i) {
    PcOutDesc pd = enqueue_pc(S, s, v, 1.0, nullptr, 0.0);
    LAUNCH_PC_OUT(pd, S->Ps(), s, S->grid(), S->sg, pd, (const double*)nullptr, 0.0, (double*)nullptr, w, 0,
           (const double*)nullptr, S->part(PT_B), S->st);
    LAUNCH(k_dot2, S->Pv(), s, A->N, (const double*)v, (const double*)w, S->part(PT_MAIN));
    LAUNCH(k_power_step, S->Pv(), s, A->N, (const double*)S->part(PT_MAIN), S->Pv(), v, (const double*)w, S->st);
  }
  noise_end(S, s);
}

int capture(pfk_session_s* S, hipGraphExec_t* out, int what, int iters) {
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(S->s1, hipStreamCaptureModeThreadLocal));
  if (what == 0) {
    enqueue_start(S, S->s1);
  } else {
    for (int i = 0; i < iters; ++i) enqueue_iteration(S);
  }
  HIPCHK(hipStreamEndCapture(S->s1, &graph));
  hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(PFK_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return PFK_OK;
}

int launch_start(pfk_session_s* S) {
  if (S->opts.use_graph) {
    if (!S->g_start) {
      int rc = capture(S, &S->g_start, 0, 0);
      if (rc) return rc;
    }
    HIPCHK(hipGraphLaunch(S->g_start, S->s1));
  } else {
    enqueue_start(S, S->s1);
  }
  HIPCHK(hipGetLastError());
  return PFK_OK;
}

int launch_iters(pfk_session_s* S, int iters) {
  if (S->opts.use_graph) {
    if (!S->g_iter) {
      int rc = capture(S, &S->g_iter, 1, S->opts.graph_iters);
      if (rc) return rc;
    }
    const int gi = S->opts.graph_iters;
    int done = 0;
    for (; done + gi <= iters; done += gi) HIPCHK(hipGraphLaunch(S->g_iter, S->s1));
    if (done < iters) {
      if (!S->g_one) {
        int rc = capture(S, &S->g_one, 1, 1);
        if (rc) return rc;
      }
      for (; done < iters; ++done) HIPCHK(hipGraphLaunch(S->g_one, S->s1));
    }
  } else {
    for (int i = 0; i < iters; ++i) enqueue_iteration(S);
  }
  HIPCHK(hipGetLastError());
  return PFK_OK;
}

int read_state(pfk_session_s* S) {
  HIPCHK(hipMemcpyAsync(S->host_state, S->st, sizeof(SolveState), hipMemcpyDeviceToHost, S->s1));
  HIPCHK(hipStreamSynchronize(S->s1));
  return PFK_OK;
}

}  // namespace

// Session set-up.  With borrowed streams (bs1 != NULL) the session uses the
// caller's two streams and creates no streams or events of its own.
static int session_make(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                        double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes, void* stream,
                        const pfk_solve_opts* opts, hipStream_t bs1, hipStream_t bs2, pfk_session* out);

extern "C" int pfk_session_create(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                                  double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes,
                                  void* stream, const pfk_solve_opts* opts, pfk_session* out) {
  return session_make(A, B, method, b, x, rtol, maxit, mmax, workspace, ws_bytes, stream, opts, nullptr, nullptr,
                      out);
}

static int session_make(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                        double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes, void* stream,
                        const pfk_solve_opts* opts, hipStream_t bs1, hipStream_t bs2, pfk_session* out) {
  if (!out) return fail(PFK_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!A || !B || !b || !x) return fail(PFK_ERR_ARG, "null argument");
  if (B->A != A) return fail(PFK_ERR_ARG, "preconditioner was made for another operator");
  if (method < PFK_FCG || method > PFK_PIPEFCG_NAIVE) return fail(PFK_ERR_ARG, "unknown method");
  if (mmax < 1 || mmax > kNuMax) return fail(PFK_ERR_ARG, "mmax must be 1..64");
  if (maxit < 0) return fail(PFK_ERR_ARG, "maxit must be >= 0");
  if (!(rtol >= 0.0)) return fail(PFK_ERR_ARG, "rtol must be >= 0");
  if (((uintptr_t)b | (uintptr_t)x) % 16 != 0) return fail(PFK_ERR_ARG, "b and x must be 16-byte aligned");
  auto* S = new (std::nothrow) pfk_session_s();
  if (!S) return fail(PFK_ERR_OOM, "host allocation");
  S->A = A; S->B = B; S->method = method; S->b = b; S->x = x; S->rtol = rtol;
  S->maxit = maxit; S->mmax = mmax;
  pfk_default_opts(&S->opts);
  if (opts) S->opts = *opts;
  if (S->opts.graph_iters < 1) S->opts.graph_iters = 1;
  if (S->opts.truncation < 0 || S->opts.truncation > 2) {
    delete S;
    return fail(PFK_ERR_ARG, "truncation must be 0, 1 or 2");
  }
  if (S->opts.norm < 0 || S->opts.norm > 1) {
    delete S;
    return fail(PFK_ERR_ARG, "norm must be 0 (2-norm) or 1 (natural)");
  }
  if (S->opts.timestamps < 0 || S->opts.timestamps > 1) {
    delete S;
    return fail(PFK_ERR_ARG, "timestamps must be 0 or 1");
  }
  if (S->opts.side_delay < 0 || S->opts.side_delay > 10000) {
    delete S;
    return fail(PFK_ERR_ARG, "side_delay must be 0..10000");
  }
  if (S->opts.stall_window < 0) {
    delete S;
    return fail(PFK_ERR_ARG, "stall_window must be >= 0");
  }
  if (S->opts.host_sync) {
    if (method != PFK_FCG && method != PFK_GCR && method != PFK_FGMRES) {
      delete S;
      return fail(PFK_ERR_ARG, "host_sync applies to FCG, GCR and FGMRES only");
    }
    S->opts.use_graph = 0;   // the host waits inside every iteration
  }
  S->L = make_layout(A, B, method, mmax, maxit);
  S->sg = A->sg;
  S->pv = A->pv_blocks;
  if (workspace) {
    if ((uintptr_t)workspace % kAlign != 0) {
      delete S;
      return fail(PFK_ERR_ARG, "workspace must be 256-byte aligned");
    }
    if (ws_bytes < S->L.total) {
      delete S;
      return fail(PFK_ERR_ARG, "workspace too small: need " + std::to_string(S->L.total) + " bytes");
    }
    S->ws = (char*)workspace;
  } else {
    if (hipMalloc(&S->ws, S->L.total) != hipSuccess) {
      delete S;
      return fail(PFK_ERR_OOM, "workspace allocation of " + std::to_string(S->L.total) + " bytes");
    }
    S->ws_owned = true;
  }
  S->st = (SolveState*)(S->ws + S->L.state);
  S->hist = (double*)(S->ws + S->L.hist);
  S->nhist = (double*)(S->ws + S->L.nhist);
  S->tstamp = (unsigned long long*)(S->ws + S->L.tstamp);
  S->user = (hipStream_t)stream;
  if (bs1) {
    S->owns_streams = false;
    S->s1 = bs1;
    S->s2 = bs2;
    if (hipHostMalloc(&S->host_state, sizeof(SolveState), hipHostMallocDefault) != hipSuccess) {
      pfk_session_destroy(S);
      return fail(PFK_ERR_HIP, "pinned state");
    }
    *out = S;
    return PFK_OK;
  }
  if (hipStreamCreateWithFlags(&S->s1, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->s2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&S->ev_user, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&S->ev_done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(&S->host_state, sizeof(SolveState), hipHostMallocDefault) != hipSuccess) {
    pfk_session_destroy(S);
    return fail(PFK_ERR_HIP, "creating streams/events");
  }
  *out = S;
  return PFK_OK;
}

extern "C" void pfk_session_destroy(pfk_session S) {
  if (!S) return;
  if (S->s1) (void)hipStreamSynchronize(S->s1);
  if (S->g_start) (void)hipGraphExecDestroy(S->g_start);
  if (S->g_iter) (void)hipGraphExecDestroy(S->g_iter);
  if (S->g_one) (void)hipGraphExecDestroy(S->g_one);
  if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
  if (S->ev_join) (void)hipEventDestroy(S->ev_join);
  if (S->ev_user) (void)hipEventDestroy(S->ev_user);
  if (S->ev_done) (void)hipEventDestroy(S->ev_done);
  if (S->owns_streams && S->s1) (void)hipStreamDestroy(S->s1);
  if (S->owns_streams && S->s2) (void)hipStreamDestroy(S->s2);
  if (S->host_state) (void)hipHostFree(S->host_state);
  if (S->ws_owned && S->ws) (void)hipFree(S->ws);
  delete S;
}

// The shift estimate (PIPEFGMRES, when not given) and the solve's set-up
// kernels (tolerance from ||b||, x = 0 when b = 0), on S->s1.
static int session_setup(pfk_session_s* S) {
  if (S->method == PFK_PIPEFGMRES && std::isnan(S->opts.shift_sigma)) {
    // sigma estimated once per session, before the set-up
    enqueue_sigma_estimate(S, S->s1, 10);
    HIPCHK(hipGetLastError());
    int rc0 = read_state(S);
    if (rc0) return rc0;
    S->sigma = S->host_state->sigma;
  } else {
    S->sigma = std::isnan(S->opts.shift_sigma) ? 0.0 : S->opts.shift_sigma;
  }
  const bool gm = S->method == PFK_FGMRES || S->method == PFK_PIPEFGMRES;
  const int nt = session_nt(S);
  LAUNCH(k_setup, 1, S->s1, S->st, 0.0, S->maxit, S->mmax, S->opts.truncation, S->opts.force_breakdown_at,
         S->sigma, gm ? 0 : S->opts.norm, S->nhist, nt, S->opts.timestamps ? S->tstamp : nullptr,
         gm ? 0 : S->opts.stall_window);
  LAUNCH(k_dot, S->Pv(), S->s1, S->A->N, S->b, S->b, S->part(PT_A));
  LAUNCH(k_setup_tol, 1, S->s1, S->part(PT_A), S->Pv(), S->rtol, S->st, S->hist);
  LAUNCH(k_zero_if_done, S->Pv(), S->s1, S->A->N, S->x, S->st);
  S->restarts = 0;
  HIPCHK(hipGetLastError());
  return PFK_OK;
}

extern "C" int pfk_session_start(pfk_session S) {
  if (!S) return fail(PFK_ERR_ARG, "null session");
  // order after the caller's queued work
  HIPCHK(hipEventRecord(S->ev_user, S->user));
  HIPCHK(hipStreamWaitEvent(S->s1, S->ev_user, 0));
  int rc = session_setup(S);
  if (rc) return rc;
  rc = launch_start(S);
  if (rc) return rc;
  HIPCHK(hipEventRecord(S->ev_done, S->s1));
  HIPCHK(hipStreamWaitEvent(S->user, S->ev_done, 0));
  return PFK_OK;
}

extern "C" int pfk_session_iterate(pfk_session S, int iters) {
  if (!S) return fail(PFK_ERR_ARG, "null session");
  if (iters <= 0) return PFK_OK;
  HIPCHK(hipEventRecord(S->ev_user, S->user));
  HIPCHK(hipStreamWaitEvent(S->s1, S->ev_user, 0));
  int rc = launch_iters(S, iters);
  if (rc) return rc;
  HIPCHK(hipEventRecord(S->ev_done, S->s1));
  HIPCHK(hipStreamWaitEvent(S->user, S->ev_done, 0));
  return PFK_OK;
}

static int fill_info(pfk_session_s* S, int rc, pfk_solve_info* info) {
  if (!info) return rc;
  const SolveState& h = *S->host_state;
  info->iterations = h.it;
  info->restarts = S->restarts;
  info->status = rc;
  double bn = 0.0;
  info->converged = (h.status == kDone) ? 1 : 0;
  bn = h.bnorm;
  info->true_rel_resid = bn > 0.0 ? h.true_res / bn : 0.0;
  info->history_len = 0;
  info->natural_len = 0;
  info->iter_time_len = 0;
  if (info->iter_time_us && info->history_cap > 0 && S->opts.timestamps) {
    // device clock ticks -> microseconds from entry 0 (the clock's rate in kHz)
    const int n = std::min(info->history_cap, h.hist_started ? h.it + 1 : 0);
    int dev = 0, khz = 0;
    std::vector<unsigned long long> t((size_t)std::max(n, 0));
    if (n > 0 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0 &&
        hipMemcpy(t.data(), S->tstamp, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost) == hipSuccess) {
      for (int i = 0; i < n; ++i) info->iter_time_us[i] = (double)(long long)(t[i] - t[0]) * 1e3 / khz;
      info->iter_time_len = n;
    }
  }
  if (info->natural_history && info->history_cap > 0) {
    const int n = std::min(info->history_cap, h.nat_started ? h.it + 1 : 0);
    if (n > 0 && hipMemcpy(info->natural_history, S->nhist, sizeof(double) * n, hipMemcpyDeviceToHost) ==
                     hipSuccess)
      info->natural_len = n;
  }
  if (info->history && info->history_cap > 0) {
    const int n = std::min(info->history_cap, h.hist_started ? h.it + 1 : 0);
    if (n > 0 && hipMemcpy(info->history, S->hist, sizeof(double) * n, hipMemcpyDeviceToHost) == hipSuccess)
      info->history_len = n;
  }
  return rc;
}

extern "C" int pfk_session_sync(pfk_session S, pfk_solve_info* info) {
  if (!S) return fail(PFK_ERR_ARG, "null session");
  int rc = read_state(S);
  if (rc) return rc;
  const int status = S->host_state->status;
  int code = PFK_OK;
  if (status == kRunning || status == kMaxit || status == kCycleEnd) code = PFK_NOT_CONVERGED;
  if (status == kNonfinite) code = PFK_ERR_NONFINITE;
  if (status == kBreakdown0) code = PFK_ERR_BREAKDOWN;
  if (status == kBreakdown || status == kGap || status == kConverged) code = PFK_NOT_CONVERGED;
  return fill_info(S, code, info);
}

// The host loop of a full solve after its start-up has been enqueued:
// iterate in graph chunks (or direct launches), check the true residual on
// convergence, restart on breakdown or residual gap; then the true residual
// at exit.  Returns a HIP/argument error (rc) or PFK_OK with *code set.
static int solve_loop(pfk_session_s* S, int* code_out) {
  int code = PFK_NOT_CONVERGED;
  int rc = PFK_OK;
  const int max_restarts = S->opts.max_restarts;
  while (rc == PFK_OK) {
    rc = read_state(S);
    if (rc) break;
    const int status = S->host_state->status;
    if (status == kRunning) {
      rc = launch_iters(S, S->opts.graph_iters);
      continue;
    }
    if (status == kConverged) {
      enqueue_true_check(S, S->s1);
      continue;
    }
    if (status == kCycleEnd) {
      // GMRES family: the restart length was reached; x = x0 + U y is in place
      if (S->host_state->it >= S->maxit) { code = PFK_NOT_CONVERGED; break; }
      rc = launch_start(S);
      continue;
    }
    if (status == kDone) { code = PFK_OK; break; }
    if (status == kMaxit) { code = PFK_NOT_CONVERGED; break; }
    if (status == kNonfinite) { code = PFK_ERR_NONFINITE; break; }
    if (status == kBreakdown0) { code = PFK_ERR_BREAKDOWN; break; }
    if (status == kBreakdown || status == kGap) {
      // the restart is counted first, also when maxit ends the solve here
      if (++S->restarts > max_restarts) {
        code = status == kBreakdown ? PFK_ERR_BREAKDOWN : PFK_NOT_CONVERGED;
        break;
      }
      if (S->host_state->it >= S->maxit) { code = PFK_NOT_CONVERGED; break; }
      rc = launch_start(S);
      continue;
    }
    code = PFK_NOT_CONVERGED;
    break;
  }
  if (rc == PFK_OK) {
    // the true residual at exit (also after maxit)
    if (!S->host_state->bzero) enqueue_true_residual(S, S->s1);
    rc = read_state(S);
  }
  *code_out = code;
  return rc;
}

// The full solve: start, then the host loop above.
extern "C" int pfk_solve(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                         double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes, void* stream,
                         const pfk_solve_opts* opts, pfk_solve_info* info) {
  pfk_session S = nullptr;
  int rc = pfk_session_create(A, B, method, b, x, rtol, maxit, mmax, workspace, ws_bytes, stream, opts, &S);
  if (rc) return rc;
  rc = pfk_session_start(S);
  int code = PFK_NOT_CONVERGED;
  if (rc == PFK_OK) rc = solve_loop(S, &code);
  if (rc == PFK_OK) {
    fill_info(S, code, info);
    if (info) info->converged = (code == PFK_OK) ? 1 : 0;
  } else if (info) {
    info->status = rc;
  }
  (void)hipEventRecord(S->ev_done, S->s1);
  (void)hipStreamWaitEvent(S->user, S->ev_done, 0);
  pfk_session_destroy(S);
  return rc ? rc : code;
}

// ---------------------------------------------------------------------------
// the solve for callers that cannot allocate
// ---------------------------------------------------------------------------
// pfk_solve_noalloc's workspace: a fixed array in device memory, one copy on
// every GPU the library runs on, held until the process ends.  Host code
// never uses the symbol's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's address of `scratch`.
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PFK_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PFK_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PFK_OK;
}

// Zero n 8-byte words (a kernel, so the call can also be recorded in a graph).
__global__ void __launch_bounds__(kBlock) k_zero_words(unsigned long long* __restrict__ p, long long n) {
  for (long long e = gtid(); e < n; e += gstride()) p[e] = 0ull;
}

}  // namespace

extern "C" int pfk_solve_noalloc(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                                 double rtol, int maxit, int mmax, void* stream, const pfk_solve_opts* opts,
                                 pfk_solve_info* info) {
  if (!A || !B || !b || !x) return fail(PFK_ERR_ARG, "null argument");
  if (B->A != A) return fail(PFK_ERR_ARG, "preconditioner was made for another operator");
  if (method < PFK_FCG || method > PFK_PIPEFCG_NAIVE) return fail(PFK_ERR_ARG, "unknown method");
  if (mmax < 1 || mmax > kNuMax) return fail(PFK_ERR_ARG, "mmax must be 1..64");
  if (maxit < 0) return fail(PFK_ERR_ARG, "maxit must be >= 0");
  if (!(rtol >= 0.0)) return fail(PFK_ERR_ARG, "rtol must be >= 0");
  if (((uintptr_t)b | (uintptr_t)x) % 16 != 0) return fail(PFK_ERR_ARG, "b and x must be 16-byte aligned");
  pfk_session_s S;   // on the stack: no host or device allocation
  pfk_default_opts(&S.opts);
  if (opts) S.opts = *opts;
  if (S.opts.graph_iters < 1) S.opts.graph_iters = 1;
  if (S.opts.truncation < 0 || S.opts.truncation > 2) return fail(PFK_ERR_ARG, "truncation must be 0, 1 or 2");
  if (S.opts.norm < 0 || S.opts.norm > 1) return fail(PFK_ERR_ARG, "norm must be 0 (2-norm) or 1 (natural)");
  if (S.opts.side_delay < 0 || S.opts.side_delay > 10000) return fail(PFK_ERR_ARG, "side_delay must be 0..10000");
  if (S.opts.stall_window < 0) return fail(PFK_ERR_ARG, "stall_window must be >= 0");
  if (S.opts.timestamps)
    return fail(PFK_ERR_ARG, "timestamps are not available in the no-allocation solve (use pfk_solve)");
  if (S.opts.host_sync && method != PFK_FCG && method != PFK_GCR && method != PFK_FGMRES)
    return fail(PFK_ERR_ARG, "host_sync applies to FCG, GCR and FGMRES only");
  S.opts.use_graph = 0;   // instantiating a graph allocates: kernels are launched directly
  S.L = make_layout(A, B, method, mmax, maxit);
  if (S.L.total > kScratchBytes)
    return fail(PFK_ERR_ARG, "this solve needs " + std::to_string(S.L.total) +
                                 " bytes of workspace; the no-allocation solve has " +
                                 std::to_string(kScratchBytes) + " (use pfk_solve with a workspace)");
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  SolveState host_state{};   // the host's copy of the device state, also on the stack
  S.A = A; S.B = B; S.method = method; S.b = b; S.x = x; S.rtol = rtol;
  S.maxit = maxit; S.mmax = mmax;
  S.sg = A->sg;
  S.pv = A->pv_blocks;
  S.ws = (char*)ws;
  S.ws_owned = false;
  S.st = (SolveState*)(S.ws + S.L.state);
  S.hist = (double*)(S.ws + S.L.hist);
  S.nhist = (double*)(S.ws + S.L.nhist);
  S.tstamp = (unsigned long long*)(S.ws + S.L.tstamp);
  // one stream, the caller's: the second stream's branch runs in order on it
  S.user = S.s1 = S.s2 = (hipStream_t)stream;
  S.owns_streams = false;
  S.host_state = &host_state;
  // the array keeps the previous call's contents: the state and the histories
  // start from zero (every other part is written before it is read)
  LAUNCH(k_zero_words, 64, S.s1, (unsigned long long*)S.ws, (long long)(S.L.vec[0] / 8));
  HIPCHK(hipGetLastError());
  rc = session_setup(&S);
  if (rc == PFK_OK) rc = launch_start(&S);
  int code = PFK_NOT_CONVERGED;
  if (rc == PFK_OK) rc = solve_loop(&S, &code);
  if (rc == PFK_OK) {
    fill_info(&S, code, info);
    if (info) info->converged = (code == PFK_OK) ? 1 : 0;
  } else if (info) {
    info->status = rc;
  }
  return rc ? rc : code;
}

extern "C" int pfk_precond_apply(pfk_precond B, const double* v, double* y, void* stream) {
  if (!B || !v || !y) return fail(PFK_ERR_ARG, "null argument");
  if (((uintptr_t)v | (uintptr_t)y) % 16 != 0) return fail(PFK_ERR_ARG, "v and y must be 16-byte aligned");
  pfk_operator A = B->A;
  Layout L = make_layout(A, B, PFK_FCG, 1, 1);
  if (!B->scratch || B->scratch_bytes < L.total) {
    if (B->scratch) (void)hipFree(B->scratch);
    B->scratch = nullptr;
    if (hipMalloc(&B->scratch, L.total) != hipSuccess) return fail(PFK_ERR_OOM, "preconditioner scratch");
    B->scratch_bytes = L.total;
  }
  pfk_session_s S;
  S.A = A; S.B = B; S.ws = B->scratch; S.L = L; S.mmax = 1;
  S.sg = A->sg; S.pv = A->pv_blocks;
  S.st = (SolveState*)(S.ws + L.state);
  if (B->kind == PFK_PC_NOISY) S.noise_draw = B->draws++;
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(k_set_running, 1, s, S.st, session_nt(&S));
  PcOutDesc pd = enqueue_pc(&S, s, v, 1.0, nullptr, 0.0);
  LAUNCH(k_pc_write, A->pv_blocks, s, A->N, pd, y, S.st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return PFK_OK;
}

extern "C" int pfk_session_profile(pfk_session S, int iters, int cap, const char** names, double* total_ms,
                                   int* launches) {
  if (!S || iters < 0 || cap < 0) return fail(PFK_ERR_ARG, "bad argument");
  HIPCHK(hipEventRecord(S->ev_user, S->user));
  HIPCHK(hipStreamWaitEvent(S->s1, S->ev_user, 0));
  KernelProfiler prof;
  g_prof = &prof;
  for (int i = 0; i < iters; ++i) enqueue_iteration(S);
  g_prof = nullptr;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(S->s1));
  std::vector<const char*> nm;
  std::vector<double> ms;
  std::vector<int> cnt;
  for (const auto& r : prof.recs) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    size_t c = 0;
    while (c < nm.size() && std::strcmp(nm[c], r.name) != 0) ++c;
    if (c == nm.size()) {
      nm.push_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[c] += t;
    cnt[c] += 1;
  }
  const int n = (int)nm.size();
  for (int c = 0; c < n && c < cap; ++c) {
    if (names) names[c] = nm[c];
    if (total_ms) total_ms[c] = ms[c];
    if (launches) launches[c] = cnt[c];
  }
  HIPCHK(hipEventRecord(S->ev_done, S->s1));
  HIPCHK(hipStreamWaitEvent(S->user, S->ev_done, 0));
  return n;
}

extern "C" int pfk_estimate_sigma(pfk_operator A, pfk_precond B, int its, double* sigma, void* stream) {
  if (!A || !B || !sigma || its < 1) return fail(PFK_ERR_ARG, "bad argument");
  if (B->A != A) return fail(PFK_ERR_ARG, "preconditioner was made for another operator");
  Layout L = make_layout(A, B, PFK_FCG, 1, 1);
  char* ws = nullptr;
  if (hipMalloc(&ws, L.total) != hipSuccess) return fail(PFK_ERR_OOM, "sigma estimate workspace");
  pfk_session_s S;
  S.A = A; S.B = B; S.ws = ws; S.L = L; S.mmax = 1;
  S.sg = A->sg; S.pv = A->pv_blocks;
  S.st = (SolveState*)(S.ws + L.state);
  hipStream_t s = (hipStream_t)stream;
  enqueue_sigma_estimate(&S, s, its);
  SolveState* h = nullptr;
  int rc = PFK_OK;
  if (hipGetLastError() != hipSuccess || hipHostMalloc(&h, sizeof(SolveState), hipHostMallocDefault) != hipSuccess ||
      hipMemcpyAsync(h, S.st, sizeof(SolveState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    rc = fail(PFK_ERR_HIP, "sigma estimate");
  } else {
    *sigma = h->sigma;
  }
  if (h) (void)hipHostFree(h);
  (void)hipFree(ws);
  return rc;
}

// ---------------------------------------------------------------------------
// launch geometry and its autotuner
// ---------------------------------------------------------------------------
namespace {
constexpr int kMaxLaunchBlocks = 16384;   // largest workgroup count of a stencil or vector launch

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
}  // namespace

extern "C" int pfk_operator_set_tiling(pfk_operator A, int tile_x, int stencil_target, int vector_blocks) {
  if (!A) return fail(PFK_ERR_ARG, "null operator");
  if (tile_x != 32 && tile_x != 64) return fail(PFK_ERR_ARG, "tile_x must be 32 or 64");
  if (stencil_target < 1 || stencil_target > kMaxLaunchBlocks) return fail(PFK_ERR_ARG, "stencil_target out of range");
  if (vector_blocks < 1 || vector_blocks > kMaxLaunchBlocks) return fail(PFK_ERR_ARG, "vector_blocks out of range");
  const StencilGeom sg = make_geom(A->dim, (int)A->n[0], (int)A->n[1], (int)A->n[2], tile_x, stencil_target);
  if (sg.blocks() > kMaxLaunchBlocks) return fail(PFK_ERR_ARG, "stencil launch too large");
  A->sg = sg;
  A->stencil_target = stencil_target;
  A->pv_blocks = vector_blocks;
  return PFK_OK;
}

extern "C" int pfk_operator_get_tiling(pfk_operator A, int* tile_x, int* stencil_blocks, int* vector_blocks) {
  if (!A) return fail(PFK_ERR_ARG, "null operator");
  if (tile_x) *tile_x = A->sg.tx;
  if (stencil_blocks) *stencil_blocks = A->sg.blocks();
  if (vector_blocks) *vector_blocks = A->pv_blocks;
  return PFK_OK;
}

// Time whole outer iterations of `method` with B on A for each candidate launch
// geometry (coordinate search: stencil tile shape and z-chunking first, then
// the vector kernels' workgroup count) and keep the fastest in A.  The solve
// runs from b = 1, x = 0 with rtol = 0 in library-owned memory; the window is
// filled before timing, so every timed iteration is a steady-state one.
extern "C" int pfk_operator_autotune(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int reps,
                                     void* stream, pfk_tuning* out) {
  if (!A || !B) return fail(PFK_ERR_ARG, "null argument");
  if (B->A != A) return fail(PFK_ERR_ARG, "preconditioner was made for another operator");
  if (method < PFK_FCG || method > PFK_PIPEFCG_NAIVE) return fail(PFK_ERR_ARG, "unknown method");
  if (mmax < 1 || mmax > kNuMax) return fail(PFK_ERR_ARG, "mmax must be 1..64");
  if (reps < 1) reps = 5;
  const int nx = (int)A->n[0], ny = (int)A->n[1], nz = (int)A->n[2];
  // candidates
  std::vector<StencilGeom> geoms;
  std::vector<int> targets;
  for (int tx : {64, 32})
    for (int target : {512, 1024, 2048, 4096}) {
      const StencilGeom g = make_geom(A->dim, nx, ny, nz, tx, target);
      bool dup = false;
      for (const auto& h : geoms) dup = dup || (h.tx == g.tx && h.zc == g.zc);
      if (!dup && g.blocks() <= kMaxLaunchBlocks) {
        geoms.push_back(g);
        targets.push_back(target);
      }
    }
  std::vector<int> pvs;
  const int pv_cap = std::max(1, std::min(kMaxLaunchBlocks, ceil_div(A->N, 2LL * kBlock)));
  for (int v = 64; v < pv_cap; v *= 2) pvs.push_back(v);
  pvs.push_back(pv_cap);
  int pmax = 0;
  for (const auto& g : geoms) pmax = std::max(pmax, g.blocks());
  for (int v : pvs) pmax = std::max(pmax, v);

  const StencilGeom sg0 = A->sg;
  const int pv0 = A->pv_blocks;
  double* bx = nullptr;
  if (hipMalloc(&bx, 2 * sizeof(double) * (size_t)((A->N + 31) / 32 * 32)) != hipSuccess)
    return fail(PFK_ERR_OOM, "autotune vectors");
  double* b = bx;
  double* x = bx + (A->N + 31) / 32 * 32;
  hipStream_t us = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill, dim3(A->pv_blocks), dim3(kBlock), 0, us, A->N, b, 1.0);
  hipLaunchKernelGGL(k_fill, dim3(A->pv_blocks), dim3(kBlock), 0, us, A->N, x, 0.0);
  pfk_solve_opts o;
  pfk_default_opts(&o);
  o.use_graph = 0;
  // GMRES types are timed over whole cycles from a restart (a column's cost
  // grows with its index); CG/CR types over steady-state iterations
  const bool gm = method == PFK_FGMRES || method == PFK_PIPEFGMRES;
  if (gm) reps = mmax;
  if (method == PFK_PIPEFGMRES) {
    double sig = 0.0;
    const int r0 = pfk_estimate_sigma(A, B, 10, &sig, stream);
    if (r0) {
      (void)hipFree(bx);
      return r0;
    }
    o.shift_sigma = sig;
  }
  const int warm = gm ? 0 : mmax + 2;
  const int maxit = warm + (int)(geoms.size() + pvs.size() + 2) * (reps + mmax + 2) + 16;
  pfk_session S = nullptr;
  int rc = pfk_session_create(A, B, method, b, x, 0.0, maxit, mmax, nullptr, 0, stream, &o, &S);
  if (rc) {
    (void)hipFree(bx);
    return rc;
  }
  // re-lay the workspace so every candidate's partial sums fit
  (void)hipFree(S->ws);
  S->L = make_layout(A, B, method, mmax, maxit, pmax);
  if (hipMalloc(&S->ws, S->L.total) != hipSuccess) {
    S->ws = nullptr;
    pfk_session_destroy(S);
    (void)hipFree(bx);
    return fail(PFK_ERR_OOM, "autotune workspace");
  }
  S->st = (SolveState*)(S->ws + S->L.state);
  S->hist = (double*)(S->ws + S->L.hist);
  S->nhist = (double*)(S->ws + S->L.nhist);
  S->tstamp = (unsigned long long*)(S->ws + S->L.tstamp);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 0.0, dflt = 0.0;
  int count = 0;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pfk_session_destroy(S);
    (void)hipFree(bx);
  };
  // mean time of `reps` iterations with the session's current geometry
  // (restarted from x if the solve stopped, e.g. at a GMRES cycle end)
  auto time_iters = [&](double* ms) -> int {
    int r = read_state(S);
    if (r) return r;
    if (gm || S->host_state->status != kRunning || S->host_state->it + reps + 2 >= maxit) {
      r = pfk_session_start(S);
      if (r) return r;
      for (int i = 0; i < warm; ++i) enqueue_iteration(S);
    }
    HIPCHK(hipEventRecord(e0, S->s1));
    for (int i = 0; i < reps; ++i) enqueue_iteration(S);
    HIPCHK(hipEventRecord(e1, S->s1));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / reps;
    ++count;
    return PFK_OK;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(PFK_ERR_HIP, "autotune events");
  }
  rc = pfk_session_start(S);
  if (!rc) {
    for (int i = 0; i < warm; ++i) enqueue_iteration(S);
    rc = time_iters(&dflt);   // the geometry the operator had
  }
  StencilGeom best_sg = sg0;
  int best_target = A->stencil_target;
  int best_pv = pv0;
  best = dflt;
  for (size_t c = 0; !rc && c < geoms.size(); ++c) {
    S->sg = geoms[c];
    double t = 0.0;
    rc = time_iters(&t);
    if (!rc && t < best) { best = t; best_sg = geoms[c]; best_target = targets[c]; }
  }
  S->sg = best_sg;
  for (size_t c = 0; !rc && c < pvs.size(); ++c) {
    S->pv = pvs[c];
    double t = 0.0;
    rc = time_iters(&t);
    if (!rc && t < best) { best = t; best_pv = pvs[c]; }
  }
  if (!rc) HIPCHK(hipStreamSynchronize(S->s1));
  cleanup();
  if (rc) return rc;
  A->sg = best_sg;
  A->stencil_target = best_target;
  A->pv_blocks = best_pv;
  if (out) {
    out->tile_x = best_sg.tx;
    out->stencil_target = best_target;
    out->stencil_blocks = best_sg.blocks();
    out->vector_blocks = best_pv;
    out->ms_per_iteration = best;
    out->ms_default = dflt;
    out->candidates = count;
  }
  return PFK_OK;
}

// ---------------------------------------------------------------------------
// batches: many independent systems advanced by shared launches
// ---------------------------------------------------------------------------
struct pfk_batch_s {
  int method = 0, mmax = 0;
  pfk_solve_opts opts{};
  hipStream_t user = nullptr, s1 = nullptr, s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_user = nullptr, ev_done = nullptr;
  int dim = 0, fp32 = -1, pc_kind = -1;   // shared by every member (fixed by the first one added)
  int pc_k = -1;                          // inner steps, shared when the inner solve is global
  struct Member {
    pfk_session S = nullptr;
    int state = 0;     // 0 free, 1 running, 2 finished
    int code = 0;      // pfk_status once finished
  };
  std::vector<Member> mem;
  // device tables of the running members (rebuilt when the running set changes)
  std::vector<int> rows;                  // member index of each table row
  BSys* d_sys = nullptr;
  int* d_off = nullptr;                   // kBpCount arrays of (rows + 1) range starts
  int* d_stat = nullptr;                  // 2 ints per row: status, iteration
  int* h_stat = nullptr;                  // pinned copy
  int cap_rows = 0;
  int tot[kBpCount] = {};
  int stale = 0;                          // vector workgroups of table rows whose member ended
  bool dirty = true;
  hipGraphExec_t graph = nullptr;
  GridBarrier* bar = nullptr;             // persistent form: grid barrier state
  GridBarrier* h_bar = nullptr;           // pinned initial value of it
  long long barrier_limit = kBarrierSpins;
  int coop_grid = 0;                      // its workgroup count (0: not yet sized)
};

namespace {

bool batch_method_ok(int m) { return m == PFK_PIPEFCG || m == PFK_FCG || m == PFK_PIPEFGMRES; }

// The table record of one member (its session's buffers and geometry).
BSys make_bsys(const pfk_session_s* S) {
  const pfk_operator_s* A = S->A;
  BSys d{};
  d.N = A->N;
  d.g = A->grid();
  if (A->eta_bf16) d.gm = A->grid_mixed();
  d.sg = S->sg;
  d.Pv = S->Pv();
  d.Ps = S->Ps();
  d.bj_wy = (int)((A->n[1] + kBjEdge - 1) / kBjEdge);
  if (A->dim == 3) {
    d.bj_wx = (int)((A->n[0] + 2 * kBjEdge - 1) / (2 * kBjEdge));
    d.bj_n = d.bj_wx * d.bj_wy * (int)((A->n[2] + kBjEdge - 1) / kBjEdge);
  } else {
    d.bj_wx = (int)((A->n[0] + 4 * kBjEdge - 1) / (4 * kBjEdge));
    d.bj_n = d.bj_wx * d.bj_wy;
  }
  d.pc_k = S->B->k;
  switch (S->method) {
    case PFK_PIPEFCG: d.pd = pc_out_desc(S, S->vec(V_W), 1.0, S->vec(V_R), -1.0); break;
    case PFK_FCG: d.pd = pc_out_desc(S, S->vec(V_R), 1.0, nullptr, 0.0); break;
    default: d.pd = pc_out_desc(S, S->vec(V_M), 1.0, nullptr, 0.0); break;   // PIPEFGMRES: B(zbar)
  }
  d.P = S->win(W_P);
  d.S = S->win(W_S);
  d.Q = S->win(W_Q);
  d.Z = S->win(W_Z);
  d.pc_pbase = S->win(W_PCP).base;
  d.pc_ldp = S->L.ld;
  d.pc_q = S->vec(V_PC_Q);
  d.pc_rho = S->vec(V_PC_RHO);
  d.part_pc0 = S->part(PT_PC0);
  d.part_pc1 = S->part(PT_PC1);
  d.x = S->x;
  d.r = S->vec(V_R);
  d.u = S->vec(V_U);
  d.w = S->vec(V_W);
  d.m = S->vec(V_M);
  d.n = S->vec(V_N);
  d.z = S->vec(V_Z);
  d.x0 = S->vec(V_X0);
  d.part_main = S->part(PT_MAIN);
  d.part_a = S->part(PT_A);
  d.part_b = S->part(PT_B);
  d.st = S->st;
  d.hist = S->hist;
  return d;
}

int batch_rebuild(pfk_batch_s* T) {
  HIPCHK(hipStreamSynchronize(T->s1));   // in-flight launches read the old tables
  if (T->graph) {
    (void)hipGraphExecDestroy(T->graph);
    T->graph = nullptr;
  }
  T->rows.clear();
  for (int i = 0; i < (int)T->mem.size(); ++i)
    if (T->mem[i].state == 1) T->rows.push_back(i);
  const int n = (int)T->rows.size();
  if (n > T->cap_rows) {
    if (T->d_sys) (void)hipFree(T->d_sys);
    if (T->d_off) (void)hipFree(T->d_off);
    if (T->d_stat) (void)hipFree(T->d_stat);
    if (T->h_stat) (void)hipHostFree(T->h_stat);
    T->d_sys = nullptr; T->d_off = nullptr; T->d_stat = nullptr; T->h_stat = nullptr;
    T->cap_rows = 0;
    if (hipMalloc(&T->d_sys, sizeof(BSys) * n) != hipSuccess ||
        hipMalloc(&T->d_off, sizeof(int) * kBpCount * (n + 1)) != hipSuccess ||
        hipMalloc(&T->d_stat, sizeof(int) * 2 * n) != hipSuccess ||
        hipHostMalloc(&T->h_stat, sizeof(int) * 2 * n, hipHostMallocDefault) != hipSuccess)
      return fail(PFK_ERR_OOM, "batch tables");
    T->cap_rows = n;
  }
  std::vector<BSys> sys(n);
  std::vector<int> off((size_t)kBpCount * (n + 1), 0);
  for (int p = 0; p < kBpCount; ++p) T->tot[p] = 0;
  for (int r = 0; r < n; ++r) {
    sys[r] = make_bsys(T->mem[T->rows[r]].S);
    const int cnt[kBpCount] = {sys[r].Pv, sys[r].Ps, sys[r].bj_n, 1};
    for (int p = 0; p < kBpCount; ++p) {
      off[(size_t)p * (n + 1) + r] = T->tot[p];
      T->tot[p] += p == kBpOne ? 1 : (cnt[p] + 7) / 8 * 8;   // ranges start at multiples of 8
    }
  }
  for (int p = 0; p < kBpCount; ++p) off[(size_t)p * (n + 1) + n] = T->tot[p];
  if (n > 0) {
    HIPCHK(hipMemcpy(T->d_sys, sys.data(), sizeof(BSys) * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(T->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
  }
  T->stale = 0;
  T->dirty = false;
  return PFK_OK;
}

template <class T>
void batch_block_pc(pfk_batch_s* Tb, const int* off, int n) {
  hipStream_t s1 = Tb->s1;
  if (Tb->dim == 3) LAUNCH((kb_block_pcg<T, 1>), Tb->tot[kBpBlk], s1, Tb->d_sys, off, n);
  else LAUNCH((kb_block_pcg<T, 0>), Tb->tot[kBpBlk], s1, Tb->d_sys, off, n);
}

// The global inner solves of every member, phase by phase as a single solve
// launches them (os: stencil ranges, ov: vector ranges).
template <class T>
void batch_inner_pcg(pfk_batch_s* Tb, const int* os, const int* ov, int n) {
  hipStream_t s1 = Tb->s1;
  LAUNCH((kb_pcg_a1<T>), Tb->tot[kBpSten], s1, Tb->d_sys, os, n);
  for (int j = 1; j < Tb->pc_k; ++j) {
    LAUNCH((kb_pcg_b<T>), Tb->tot[kBpVec], s1, Tb->d_sys, ov, n, j);
    LAUNCH((kb_pcg_a<T>), Tb->tot[kBpSten], s1, Tb->d_sys, os, n, j);
  }
}
template <class T>
void batch_inner_gmres(pfk_batch_s* Tb, const int* os, int n) {
  hipStream_t s1 = Tb->s1;
#define PFK_KBGF(J)                                                                           \
  do {                                                                                        \
    if (j + 1 == Tb->pc_k) LAUNCH((kb_gmpc_fused<T, J, true>), Tb->tot[kBpSten], s1, Tb->d_sys, os, n, j); \
    else LAUNCH((kb_gmpc_fused<T, J, false>), Tb->tot[kBpSten], s1, Tb->d_sys, os, n, j);                   \
  } while (0)
  for (int j = 0; j < Tb->pc_k; ++j) {
    switch (j) {
      case 0: PFK_KBGF(0); break;
      case 1: PFK_KBGF(1); break;
      case 2: PFK_KBGF(2); break;
      case 3: PFK_KBGF(3); break;
      case 4: PFK_KBGF(4); break;
      default: PFK_KBGF(kGfFixed + 1); break;
    }
  }
#undef PFK_KBGF
  LAUNCH(kb_gmpc_finish, n, s1, Tb->d_sys, n);
}

// The batched consumer of the inner solve's output, instantiated per inner
// kind and storage (all members share them).
void launch_batch_pc_out(pfk_batch_s* T, const int* os, int n, int pipefcg) {
  hipStream_t s1 = T->s1;
  const int K = T->pc_kind;
  if (K == kPcBlockPcg) {
    if (T->fp32) LAUNCH((kb_apply_pc_out<kPcBlockPcg, 1>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
    else LAUNCH((kb_apply_pc_out<kPcBlockPcg, 0>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
  } else if (K == kPcJacobiPcg) {
    if (T->fp32) LAUNCH((kb_apply_pc_out<kPcJacobiPcg, 1>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
    else LAUNCH((kb_apply_pc_out<kPcJacobiPcg, 0>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
  } else if (K == kPcJacobiGmres && T->fp32 && T->pc_k <= kGmRaw) {
    LAUNCH((kb_apply_pc_out<kPcJacobiGmres, 1>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
  } else {
    LAUNCH((kb_apply_pc_out<-1, 0>), T->tot[kBpSten], s1, T->d_sys, os, n, pipefcg);
  }
}

// One outer iteration of every running member.
void enqueue_batch_iteration(pfk_batch_s* T) {
  const int n = (int)T->rows.size();
  const int* ov = T->d_off + kBpVec * (n + 1);
  const int* os = T->d_off + kBpSten * (n + 1);
  const int* ob = T->d_off + kBpBlk * (n + 1);
  hipStream_t s1 = T->s1, s2 = T->s2;
  auto pc = [&]() {
    switch (T->pc_kind) {
      case kPcBlockPcg:
        if (T->fp32) batch_block_pc<float>(T, ob, n);
        else batch_block_pc<double>(T, ob, n);
        break;
      case kPcJacobiPcg:
        if (T->fp32) batch_inner_pcg<float>(T, os, ov, n);
        else batch_inner_pcg<double>(T, os, ov, n);
        break;
      case kPcJacobiGmres:
        if (T->fp32) batch_inner_gmres<float>(T, os, n);
        else batch_inner_gmres<double>(T, os, n);
        break;
      default:
        break;   // NONE, JACOBI: B(v) is evaluated by its consumer
    }
  };
  switch (T->method) {
    case PFK_PIPEFCG:
      LAUNCH(kb_pipefcg_update, T->tot[kBpVec], s1, T->d_sys, ov, n);
      (void)hipEventRecord(T->ev_fork, s1);
      (void)hipStreamWaitEvent(s2, T->ev_fork, 0);
      LAUNCH(kb_pipefcg_scalars, n, s2, T->d_sys);
      (void)hipEventRecord(T->ev_join, s2);
      pc();
      launch_batch_pc_out(T, os, n, 1);
      (void)hipStreamWaitEvent(s1, T->ev_join, 0);
      break;
    case PFK_FCG:
      LAUNCH(kb_fcg_xr, T->tot[kBpVec], s1, T->d_sys, ov, n);
      pc();
      LAUNCH(kb_fcg_multidot, T->tot[kBpVec], s1, T->d_sys, ov, n);
      LAUNCH(kb_cg_scalars1, n, s1, T->d_sys);
      LAUNCH(kb_fcg_maxpy, T->tot[kBpVec], s1, T->d_sys, ov, n);
      LAUNCH(kb_fcg_apply, T->tot[kBpSten], s1, T->d_sys, os, n);
      LAUNCH(kb_cg_scalars2, n, s1, T->d_sys);
      break;
    default:   // PIPEFGMRES
      LAUNCH(kb_pgm_update, T->tot[kBpVec], s1, T->d_sys, ov, n);
      (void)hipEventRecord(T->ev_fork, s1);
      (void)hipStreamWaitEvent(s2, T->ev_fork, 0);
      LAUNCH(kb_pgm_scalars, n, s2, T->d_sys);
      (void)hipEventRecord(T->ev_join, s2);
      pc();
      launch_batch_pc_out(T, os, n, 0);
      (void)hipStreamWaitEvent(s1, T->ev_join, 0);
      LAUNCH(kb_gm_update_x, T->tot[kBpVec], s1, T->d_sys, ov, n);
      break;
  }
}

// The persistent kernel for this batch's method / inner solve / dimension.
using KpFn = void (*)(const BSys*, const int*, int, int, int, int, int, GridBarrier*);
template <int M>
KpFn kp_pick(int pc, int d3) {
  if (pc == 0) return d3 ? (KpFn)kp_batch<M, 0, 1> : (KpFn)kp_batch<M, 0, 0>;
  if (pc == 1) return d3 ? (KpFn)kp_batch<M, 1, 1> : (KpFn)kp_batch<M, 1, 0>;
  return d3 ? (KpFn)kp_batch<M, 2, 1> : (KpFn)kp_batch<M, 2, 0>;
}

KpFn kp_kernel(const pfk_batch_s* T) {
  const int pc = T->pc_kind == kPcBlockPcg ? (T->fp32 ? 2 : 1) : 0;
  const int d3 = T->dim == 3;
  if (T->method == PFK_PIPEFCG) return kp_pick<PFK_PIPEFCG>(pc, d3);
  if (T->method == PFK_FCG) return kp_pick<PFK_FCG>(pc, d3);
  return kp_pick<PFK_PIPEFGMRES>(pc, d3);
}

// `iters` iterations of every running member in one cooperative launch.  The
// grid holds as many workgroups as can be resident at once (a multiple of 8,
// so a work item and its workgroup sit on the same XCD), capped by the work.
int batch_persistent(pfk_batch_s* T, int iters) {
  KpFn fn = kp_kernel(T);
  if (!T->bar) {
    HIPCHK(hipMalloc(&T->bar, sizeof(GridBarrier)));
    HIPCHK(hipHostMalloc(&T->h_bar, sizeof(GridBarrier), hipHostMallocDefault));
  }
  int dev = 0, ncu = 0, per_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBlock, 0));
  const int most = std::max(T->tot[kBpVec], std::max(T->tot[kBpSten], T->tot[kBpBlk]));
  int G = std::min(per_cu * ncu, std::max(8, (most + 7) / 8 * 8));
  G = G / 8 * 8;
  if (G < 8) return fail(PFK_ERR_HIP, "persistent launch: no resident workgroups");
  T->coop_grid = G;
  HIPCHK(hipStreamSynchronize(T->s1));   // the pinned initial value is reused by every launch
  std::memset(T->h_bar, 0, sizeof(GridBarrier));
  T->h_bar->limit = T->barrier_limit;
  HIPCHK(hipMemcpyAsync(T->bar, T->h_bar, sizeof(GridBarrier), hipMemcpyHostToDevice, T->s1));
  const int n = (int)T->rows.size();
  const BSys* sys = T->d_sys;
  const int* off = T->d_off;
  int tv = T->tot[kBpVec], ts = T->tot[kBpSten], tb = T->tot[kBpBlk];
  void* args[] = {(void*)&sys, (void*)&off, (void*)&n, (void*)&tv, (void*)&ts, (void*)&tb, (void*)&iters,
                  (void*)&T->bar};
  HIPCHK(hipLaunchCooperativeKernel((const void*)fn, dim3(G), dim3(kBlock), args, 0, T->s1));
  return PFK_OK;
}

}  // namespace

extern "C" void pfk_batch_destroy(pfk_batch T) {
  if (!T) return;
  if (T->s1) (void)hipStreamSynchronize(T->s1);
  for (auto& m : T->mem)
    if (m.S) pfk_session_destroy(m.S);
  if (T->graph) (void)hipGraphExecDestroy(T->graph);
  if (T->d_sys) (void)hipFree(T->d_sys);
  if (T->d_off) (void)hipFree(T->d_off);
  if (T->d_stat) (void)hipFree(T->d_stat);
  if (T->h_stat) (void)hipHostFree(T->h_stat);
  if (T->bar) (void)hipFree(T->bar);
  if (T->h_bar) (void)hipHostFree(T->h_bar);
  for (hipEvent_t e : {T->ev_fork, T->ev_join, T->ev_user, T->ev_done})
    if (e) (void)hipEventDestroy(e);
  if (T->s1) (void)hipStreamDestroy(T->s1);
  if (T->s2) (void)hipStreamDestroy(T->s2);
  delete T;
}

extern "C" int pfk_batch_create(pfk_method method, int mmax, int capacity, void* stream,
                                const pfk_solve_opts* opts, pfk_batch* out) {
  if (!out) return fail(PFK_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!batch_method_ok(method)) return fail(PFK_ERR_ARG, "batches run PIPEFCG, FCG or PIPEFGMRES");
  if (mmax < 1 || mmax > kNuMax) return fail(PFK_ERR_ARG, "mmax must be 1..64");
  if (capacity < 1 || capacity > 4096) return fail(PFK_ERR_ARG, "capacity must be 1..4096");
  auto* T = new (std::nothrow) pfk_batch_s();
  if (!T) return fail(PFK_ERR_OOM, "host allocation");
  T->method = method;
  T->mmax = mmax;
  pfk_default_opts(&T->opts);
  if (opts) T->opts = *opts;
  if (T->opts.graph_iters < 1) T->opts.graph_iters = 1;
  if (T->opts.host_sync) {
    delete T;
    return fail(PFK_ERR_ARG, "host_sync does not apply to batches");
  }
  if (T->opts.persistent < 0 || T->opts.persistent > 1) {
    delete T;
    return fail(PFK_ERR_ARG, "persistent must be 0 or 1");
  }
  T->user = (hipStream_t)stream;
  T->mem.resize(capacity);
  if (hipStreamCreateWithFlags(&T->s1, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&T->s2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&T->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&T->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&T->ev_user, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&T->ev_done, hipEventDisableTiming) != hipSuccess) {
    pfk_batch_destroy(T);
    return fail(PFK_ERR_HIP, "creating streams/events");
  }
  *out = T;
  return PFK_OK;
}

extern "C" int pfk_batch_add(pfk_batch T, pfk_operator A, pfk_precond B, const double* b, double* x, double rtol,
                             int maxit, void* workspace, size_t ws_bytes, int* slot) {
  if (!T || !A || !B || !slot) return fail(PFK_ERR_ARG, "null argument");
  *slot = -1;
  const int kind = B->kind;
  if (kind == PFK_PC_NOISY) return fail(PFK_ERR_ARG, "batches do not take the noisy preconditioner");
  const bool global_inner = kind == kPcJacobiPcg || kind == kPcJacobiGmres;
  if (global_inner && T->opts.persistent)
    return fail(PFK_ERR_ARG, "the persistent form takes the NONE, JACOBI or BLOCK_JACOBI_PCG preconditioner");
  const int fp32 = (kind == kPcBlockPcg || global_inner) && B->prec == PFK_FP32_BF16COEF;
  if (T->pc_kind >= 0 && (T->pc_kind != kind || T->fp32 != fp32 || T->dim != A->dim))
    return fail(PFK_ERR_ARG, "every member of a batch has the same dimension, preconditioner kind and precision");
  if (global_inner && T->pc_kind >= 0 && T->pc_k != B->k)
    return fail(PFK_ERR_ARG, "every member of a batch has the same number of inner steps");
  int s = -1;
  for (int i = 0; i < (int)T->mem.size() && s < 0; ++i)
    if (T->mem[i].state == 0) s = i;
  if (s < 0) return fail(PFK_ERR_ARG, "batch is full");
  pfk_session S = nullptr;
  int rc = session_make(A, B, (pfk_method)T->method, b, x, rtol, maxit, T->mmax, workspace, ws_bytes, T->user,
                        &T->opts, T->s1, T->s2, &S);
  if (rc) return rc;
  S->nt_scale = (int)T->mem.size();
  // order after the caller's queued work, then the set-up and the start-up
  HIPCHK(hipEventRecord(T->ev_user, T->user));
  HIPCHK(hipStreamWaitEvent(T->s1, T->ev_user, 0));
  rc = session_setup(S);
  if (rc) {
    pfk_session_destroy(S);
    return rc;
  }
  enqueue_start(S, T->s1);
  HIPCHK(hipGetLastError());
  T->pc_kind = kind;
  T->fp32 = fp32;
  T->dim = A->dim;
  T->pc_k = B->k;
  T->mem[s].S = S;
  T->mem[s].state = 1;
  T->mem[s].code = PFK_NOT_CONVERGED;
  T->dirty = true;
  *slot = s;
  return PFK_OK;
}

namespace {

// `iters` iterations of every running member.  With `join` the batch stream
// first waits for the caller's stream and the caller's stream then waits for
// the batch (the ordering every stream-taking call of the ABI gives); the
// server steps its batches without it, so batches of different methods run
// side by side instead of each waiting for the previous one through the
// caller's stream.
int batch_step(pfk_batch_s* T, int iters, bool join) {
  if (iters <= 0) return PFK_OK;
  if (T->dirty) {
    int rc = batch_rebuild(T);
    if (rc) return rc;
  }
  if (T->rows.empty()) return PFK_OK;
  if (join) {
    HIPCHK(hipEventRecord(T->ev_user, T->user));
    HIPCHK(hipStreamWaitEvent(T->s1, T->ev_user, 0));
  }
  if (T->opts.persistent) {
    int rc = batch_persistent(T, iters);
    if (rc) return rc;
    if (join) {
      HIPCHK(hipEventRecord(T->ev_done, T->s1));
      HIPCHK(hipStreamWaitEvent(T->user, T->ev_done, 0));
    }
    return PFK_OK;
  }
  const int gi = T->opts.graph_iters;
  int done = 0;
  if (T->opts.use_graph && iters >= gi) {
    if (!T->graph) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(T->s1, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < gi; ++i) enqueue_batch_iteration(T);
      HIPCHK(hipStreamEndCapture(T->s1, &g));
      hipError_t e = hipGraphInstantiate(&T->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(PFK_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    for (; done + gi <= iters; done += gi) HIPCHK(hipGraphLaunch(T->graph, T->s1));
  }
  for (; done < iters; ++done) enqueue_batch_iteration(T);
  HIPCHK(hipGetLastError());
  if (join) {
    HIPCHK(hipEventRecord(T->ev_done, T->s1));
    HIPCHK(hipStreamWaitEvent(T->user, T->ev_done, 0));
  }
  return PFK_OK;
}

}  // namespace

extern "C" int pfk_batch_step(pfk_batch T, int iters) {
  if (!T) return fail(PFK_ERR_ARG, "null batch");
  return batch_step(T, iters, true);
}

// Collect the members' states and act on them as a single solve's host loop
// does: a recurred convergence gets its true-residual check, a GMRES cycle end
// or a breakdown/residual gap a restart from x (restarts and iterations
// bounded), anything final ends the member.  Synchronises the batch stream.
extern "C" int pfk_batch_poll(pfk_batch T, int* finished, int cap, int* nfinished, int* nrunning) {
  if (!T) return fail(PFK_ERR_ARG, "null batch");
  if (nfinished) *nfinished = 0;
  if (T->dirty) {
    int rc = batch_rebuild(T);
    if (rc) return rc;
  }
  const int n = (int)T->rows.size();
  int nf = 0, nr = 0;
  if (n > 0) {
    LAUNCH(kb_gather_status, (n + kBlock - 1) / kBlock, T->s1, (const BSys*)T->d_sys, n, T->d_stat);
    HIPCHK(hipMemcpyAsync(T->h_stat, T->d_stat, sizeof(int) * 2 * n, hipMemcpyDeviceToHost, T->s1));
    HIPCHK(hipStreamSynchronize(T->s1));
  }
  if (T->bar) {
    GridBarrier hb{};
    HIPCHK(hipMemcpy(&hb, T->bar, sizeof(GridBarrier), hipMemcpyDeviceToHost));
    if (hb.abort) return fail(PFK_ERR_HIP, "persistent launch: a grid barrier timed out");
  }
  for (int r = 0; r < n; ++r) {
    auto& mb = T->mem[T->rows[r]];
    if (mb.state != 1) continue;   // ended at an earlier poll; its row waits for the next rebuild
    pfk_session_s* S = mb.S;
    const int status = T->h_stat[2 * r], it = T->h_stat[2 * r + 1];
    bool ended = false;
    int code = PFK_NOT_CONVERGED;
    switch (status) {
      case kRunning: break;
      case kConverged: enqueue_true_check(S, T->s1); break;
      case kDone: ended = true; code = PFK_OK; break;
      case kMaxit: ended = true; break;
      case kNonfinite: ended = true; code = PFK_ERR_NONFINITE; break;
      case kBreakdown0: ended = true; code = PFK_ERR_BREAKDOWN; break;
      case kCycleEnd:
        if (it >= S->maxit) ended = true;
        else enqueue_start(S, T->s1);
        break;
      case kBreakdown:
      case kGap:
        // the restart is counted first, also when maxit ends the member here
        if (++S->restarts > S->opts.max_restarts) {
          ended = true;
          code = status == kBreakdown ? PFK_ERR_BREAKDOWN : PFK_NOT_CONVERGED;
        } else if (it >= S->maxit) {
          ended = true;
        } else {
          enqueue_start(S, T->s1);
        }
        break;
      default: ended = true; break;
    }
    if (ended) {
      // the true residual at exit (already known after a converged check)
      if (status != kDone) enqueue_true_residual(S, T->s1);
      mb.state = 2;
      mb.code = code;
      // Its device status is final (not kRunning), so every later launch
      // returns at once for its row: the tables and the captured graph stay
      // valid.  They are rebuilt once ended rows hold half of the vector
      // workgroups, not at every retirement (a rebuild synchronises the batch
      // and re-instantiates its graph).
      T->stale += (S->Pv() + 7) / 8 * 8;
      if (2 * T->stale >= T->tot[kBpVec]) T->dirty = true;
      if (finished && nf < cap) finished[nf] = T->rows[r];
      ++nf;
      continue;
    }
    ++nr;
  }
  HIPCHK(hipGetLastError());
  if (nfinished) *nfinished = nf;
  if (nrunning) *nrunning = nr;
  return PFK_OK;
}

extern "C" int pfk_batch_info(pfk_batch T, int slot, pfk_solve_info* info) {
  if (!T || slot < 0 || slot >= (int)T->mem.size() || T->mem[slot].state == 0)
    return fail(PFK_ERR_ARG, "no such member");
  auto& mb = T->mem[slot];
  int rc = read_state(mb.S);
  if (rc) return rc;
  const int code = mb.state == 2 ? mb.code : PFK_NOT_CONVERGED;
  fill_info(mb.S, code, info);
  if (info) info->converged = (mb.state == 2 && code == PFK_OK) ? 1 : 0;
  return mb.state == 2 ? code : PFK_NOT_CONVERGED;
}

extern "C" int pfk_batch_set_barrier_limit(pfk_batch T, long long polls) {
  if (!T || polls < 0) return fail(PFK_ERR_ARG, "bad argument");
  T->barrier_limit = polls;
  return PFK_OK;
}

extern "C" int pfk_batch_remove(pfk_batch T, int slot) {
  if (!T || slot < 0 || slot >= (int)T->mem.size() || T->mem[slot].state == 0)
    return fail(PFK_ERR_ARG, "no such member");
  HIPCHK(hipStreamSynchronize(T->s1));
  pfk_session_destroy(T->mem[slot].S);
  T->mem[slot] = pfk_batch_s::Member{};
  T->dirty = true;
  bool any = false;
  for (auto& m : T->mem) any = any || m.state != 0;
  if (!any) { T->pc_kind = -1; T->fp32 = -1; T->dim = 0; T->pc_k = -1; }
  return PFK_OK;
}

extern "C" size_t pfk_batch_workspace_bytes(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int maxit) {
  return pfk_workspace_bytes(A, B, method, mmax, maxit);
}

extern "C" int pfk_solve_batched(int count, const pfk_operator* A, const pfk_precond* B, pfk_method method,
                                 const double* const* b, double* const* x, const double* rtol, int maxit, int mmax,
                                 void* workspace, size_t ws_bytes, void* stream, const pfk_solve_opts* opts,
                                 pfk_solve_info* infos) {
  if (count < 1 || !A || !B || !b || !x || !rtol) return fail(PFK_ERR_ARG, "null argument");
  // member i's part of a caller workspace: its own workspace size, 256-byte aligned, in order
  std::vector<size_t> part((size_t)count, 0);
  size_t need = 0;
  for (int i = 0; i < count; ++i) {
    if (!A[i] || !B[i]) return fail(PFK_ERR_ARG, "null operator or preconditioner");
    part[i] = align_up(pfk_workspace_bytes(A[i], B[i], method, mmax, maxit));
    if (part[i] == 0) return fail(PFK_ERR_ARG, "workspace size");
    need += part[i];
  }
  if (workspace && ws_bytes < need)
    return fail(PFK_ERR_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  pfk_batch T = nullptr;
  int rc = pfk_batch_create(method, mmax, count, stream, opts, &T);
  if (rc) return rc;
  std::vector<int> slot(count, -1);
  size_t off = 0;
  for (int i = 0; i < count && !rc; ++i) {
    void* w = workspace ? (void*)((char*)workspace + off) : nullptr;
    rc = pfk_batch_add(T, A[i], B[i], b[i], x[i], rtol[i], maxit, w, workspace ? part[i] : 0, &slot[i]);
    off += part[i];
  }
  int running = count;
  const int gi = T->opts.graph_iters;
  while (!rc && running > 0) {
    rc = pfk_batch_step(T, gi);
    if (!rc) rc = pfk_batch_poll(T, nullptr, 0, nullptr, &running);
  }
  int worst = PFK_OK;
  for (int i = 0; !rc && i < count; ++i) {
    const int c = pfk_batch_info(T, slot[i], infos ? &infos[i] : nullptr);
    if (c < 0 && worst >= 0) worst = c;
    else if (c > 0 && worst == PFK_OK) worst = c;
  }
  if (!rc) HIPCHK(hipEventRecord(T->ev_done, T->s1));
  if (!rc) HIPCHK(hipStreamWaitEvent(T->user, T->ev_done, 0));
  pfk_batch_destroy(T);
  return rc ? rc : worst;
}

// ---------------------------------------------------------------------------
// serving: a request queue in front of continuously refilled batches
// ---------------------------------------------------------------------------
namespace {

// Device memory for admitted requests' workspaces: freed blocks are kept and
// reused for a request of the same or slightly smaller size (within 2x).
struct WsPool {
  std::vector<std::pair<size_t, void*>> free_blocks;
  size_t held = 0;   // bytes allocated from the device (in use or cached)
  void* get(size_t bytes, size_t budget, size_t in_use) {
    int best = -1;
    for (int i = 0; i < (int)free_blocks.size(); ++i) {
      const size_t sz = free_blocks[i].first;
      if (sz >= bytes && sz <= 2 * bytes && (best < 0 || sz < free_blocks[best].first)) best = i;
    }
    if (best >= 0) {
      void* p = free_blocks[best].second;
      free_blocks.erase(free_blocks.begin() + best);
      return p;
    }
    // release cached blocks while a fresh allocation would exceed the budget
    while (!free_blocks.empty() && held + bytes > budget + 0 && held > in_use) {
      (void)hipFree(free_blocks.back().second);
      held -= free_blocks.back().first;
      free_blocks.pop_back();
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    held += bytes;
    return p;
  }
  void put(void* p, size_t bytes) { free_blocks.push_back({bytes, p}); }
  void release_all() {
    for (auto& b : free_blocks) (void)hipFree(b.second);
    free_blocks.clear();
  }
};

}  // namespace

struct pfk_server_s {
  pfk_server_config cfg{};
  void* stream = nullptr;
  struct Req {
    pfk_operator A = nullptr;
    pfk_precond B = nullptr;
    int method = 0;
    const double* b = nullptr;
    double* x = nullptr;
    double rtol = 0.0;
    int maxit = 0;
    size_t bytes = 0;       // workspace size (counts against the budget while active)
    int state = 0;          // 0 queued, 1 active, 2 finished
    int batch = -1, slot = -1;
    void* ws = nullptr;
    int code = PFK_NOT_CONVERGED;
    pfk_solve_info info{};
    std::vector<double> hist;
  };
  std::vector<Req> reqs;                      // index = request id
  std::vector<long long> queue;               // FIFO of queued ids
  size_t qhead = 0;
  struct Bt {
    int method, kind, fp32, dim, k;
    pfk_batch T;
    std::vector<long long> owner;             // request id per slot (-1 free)
    int active;
  };
  std::vector<Bt> batches;
  size_t used = 0;
  long long completed = 0;
  WsPool pool;
};

extern "C" void pfk_server_destroy(pfk_server S) {
  if (!S) return;
  for (auto& bt : S->batches) pfk_batch_destroy(bt.T);
  for (auto& r : S->reqs)
    if (r.ws) S->pool.put(r.ws, r.bytes);
  S->pool.release_all();
  delete S;
}

extern "C" int pfk_server_create(const pfk_server_config* cfg, void* stream, pfk_server* out) {
  if (!out || !cfg) return fail(PFK_ERR_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 4096) return fail(PFK_ERR_ARG, "max_active must be 1..4096");
  if (cfg->step_iters < 1) return fail(PFK_ERR_ARG, "step_iters must be >= 1");
  if (cfg->mmax < 1 || cfg->mmax > kNuMax) return fail(PFK_ERR_ARG, "mmax must be 1..64");
  if (cfg->hbm_budget == 0) return fail(PFK_ERR_ARG, "hbm_budget must be positive");
  if (cfg->stall_window < 0 || cfg->max_restarts < 0)
    return fail(PFK_ERR_ARG, "stall_window and max_restarts must be >= 0");
  auto* S = new (std::nothrow) pfk_server_s();
  if (!S) return fail(PFK_ERR_OOM, "host allocation");
  S->cfg = *cfg;
  S->stream = stream;
  *out = S;
  return PFK_OK;
}

extern "C" int pfk_server_submit(pfk_server S, pfk_operator A, pfk_precond B, pfk_method method, const double* b,
                                 double* x, double rtol, int maxit, long long* id) {
  if (!S || !A || !B || !b || !x || !id) return fail(PFK_ERR_ARG, "null argument");
  if (!batch_method_ok(method)) return fail(PFK_ERR_ARG, "requests run PIPEFCG, FCG or PIPEFGMRES");
  if (B->A != A) return fail(PFK_ERR_ARG, "preconditioner was made for another operator");
  if (B->kind == PFK_PC_NOISY) return fail(PFK_ERR_ARG, "requests do not take the noisy preconditioner");
  if (maxit < 0 || !(rtol >= 0.0)) return fail(PFK_ERR_ARG, "bad rtol or maxit");
  pfk_server_s::Req r;
  r.A = A; r.B = B; r.method = method; r.b = b; r.x = x; r.rtol = rtol; r.maxit = maxit;
  r.bytes = pfk_workspace_bytes(A, B, method, S->cfg.mmax, maxit);
  if (r.bytes == 0) return fail(PFK_ERR_ARG, "workspace size");
  if (r.bytes > S->cfg.hbm_budget) return fail(PFK_ERR_ARG, "request larger than the whole budget");
  *id = (long long)S->reqs.size();
  S->reqs.push_back(std::move(r));
  S->queue.push_back(*id);
  return PFK_OK;
}

// One scheduling round: admit queued requests in arrival order while each fits
// a batch slot and the memory budget, advance every batch with running members
// by step_iters iterations (batches run on their own streams, so their work
// overlaps), poll, and retire what ended (workspace back to the pool).
extern "C" int pfk_server_progress(pfk_server S, long long* completed, int cap, int* ncompleted) {
  if (!S) return fail(PFK_ERR_ARG, "null server");
  if (ncompleted) *ncompleted = 0;
  // admission
  while (S->qhead < S->queue.size()) {
    auto& r = S->reqs[S->queue[S->qhead]];
    const int fp32 = r.B->kind >= kPcJacobiPcg && r.B->kind <= kPcBlockPcg && r.B->prec == PFK_FP32_BF16COEF;
    int bi = -1;
    for (int i = 0; i < (int)S->batches.size() && bi < 0; ++i) {
      const auto& bt = S->batches[i];
      const bool global_inner = r.B->kind == kPcJacobiPcg || r.B->kind == kPcJacobiGmres;
      if (bt.method == r.method && bt.kind == r.B->kind && bt.fp32 == fp32 && bt.dim == r.A->dim &&
          (!global_inner || bt.k == r.B->k))
        bi = i;
    }
    if (bi < 0) {
      pfk_solve_opts o;
      pfk_default_opts(&o);
      o.graph_iters = S->cfg.step_iters;
      o.use_graph = S->cfg.launch_direct ? 0 : 1;
      o.stall_window = S->cfg.stall_window;
      if (S->cfg.max_restarts > 0) o.max_restarts = S->cfg.max_restarts;
      pfk_server_s::Bt bt{r.method, r.B->kind, fp32, r.A->dim, r.B->k, nullptr, {}, 0};
      int rc = pfk_batch_create((pfk_method)r.method, S->cfg.mmax, S->cfg.max_active, S->stream, &o, &bt.T);
      if (rc) return rc;
      bt.owner.assign(S->cfg.max_active, -1);
      S->batches.push_back(std::move(bt));
      bi = (int)S->batches.size() - 1;
    }
    auto& bt = S->batches[bi];
    if (bt.active >= S->cfg.max_active) break;            // arrival order: the head waits
    if (S->used + r.bytes > S->cfg.hbm_budget) break;
    void* ws = S->pool.get(r.bytes, S->cfg.hbm_budget, S->used);
    if (!ws) break;                                        // out of device memory: wait for retirements
    int slot = -1;
    int rc = pfk_batch_add(bt.T, r.A, r.B, r.b, r.x, r.rtol, r.maxit, ws, r.bytes, &slot);
    if (rc) {
      S->pool.put(ws, r.bytes);
      return rc;
    }
    r.ws = ws;
    r.state = 1;
    r.batch = bi;
    r.slot = slot;
    bt.owner[slot] = S->queue[S->qhead];
    ++bt.active;
    S->used += r.bytes;
    ++S->qhead;
  }
  // advance: every batch on its own streams, none waiting for another
  for (auto& bt : S->batches)
    if (bt.active > 0) {
      int rc = batch_step(bt.T, S->cfg.step_iters, false);
      if (rc) return rc;
    }
  // retire
  int nc = 0;
  std::vector<int> fin;
  for (auto& bt : S->batches) {
    if (bt.active == 0) continue;
    fin.assign(S->cfg.max_active, -1);
    int nf = 0, nr = 0;
    int rc = pfk_batch_poll(bt.T, fin.data(), (int)fin.size(), &nf, &nr);
    if (rc) return rc;
    for (int k = 0; k < nf; ++k) {
      const int slot = fin[k];
      const long long id = bt.owner[slot];
      auto& r = S->reqs[id];
      r.hist.assign((size_t)r.maxit + 1, 0.0);
      r.info.history = r.hist.data();
      r.info.history_cap = r.maxit + 1;
      r.code = pfk_batch_info(bt.T, slot, &r.info);
      rc = pfk_batch_remove(bt.T, slot);
      if (rc) return rc;
      S->pool.put(r.ws, r.bytes);
      r.ws = nullptr;
      S->used -= r.bytes;
      r.state = 2;
      bt.owner[slot] = -1;
      --bt.active;
      ++S->completed;
      if (completed && nc < cap) completed[nc] = id;
      ++nc;
    }
  }
  if (ncompleted) *ncompleted = nc;
  return PFK_OK;
}

extern "C" int pfk_server_result(pfk_server S, long long id, pfk_solve_info* info) {
  if (!S || id < 0 || id >= (long long)S->reqs.size()) return fail(PFK_ERR_ARG, "no such request");
  const auto& r = S->reqs[id];
  if (r.state != 2) return fail(PFK_ERR_ARG, "request not finished");
  if (info) {
    double* h = info->history;
    double* nh = info->natural_history;
    double* tu = info->iter_time_us;
    const int cap = info->history_cap;
    *info = r.info;
    info->history = h;
    info->natural_history = nh;
    info->natural_len = 0;
    info->iter_time_us = tu;
    info->iter_time_len = 0;
    info->history_cap = cap;
    info->history_len = 0;
    if (h && cap > 0) {
      const int n = std::min(cap, r.info.history_len);
      std::memcpy(h, r.hist.data(), sizeof(double) * n);
      info->history_len = n;
    }
  }
  return r.code;
}

extern "C" int pfk_server_stats(pfk_server S, pfk_server_status* st) {
  if (!S || !st) return fail(PFK_ERR_ARG, "null argument");
  st->queued = (long long)(S->queue.size() - S->qhead);
  st->active = 0;
  for (const auto& bt : S->batches) st->active += bt.active;
  st->completed = S->completed;
  st->bytes_in_use = S->used;
  st->bytes_held = S->pool.held;
  return PFK_OK;
}
