/*
 * pfk -- pipelined flexible Krylov solvers on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libpfk.so.  It solves A x = b with a flexible
 * (nonlinear, inner-iterative) preconditioner B, by the methods of Sanan,
 * Schnepp and May, "Pipelined, Flexible Krylov Subspace Methods":
 *   FCG (Alg. 2) and its pipelined form PIPEFCG (Alg. 8),
 *   GCR (Alg. 9) and PIPEGCR (Alg. 11),
 *   FGMRES (Alg. 13) and PIPEFGMRES (Alg. 15).
 * Each takes (A, B, b, x0) as in the paper's listings; FGMRES types also take
 * the restart length m.  Every step of the solve runs in the library's HIP
 * kernels on the GPU; the host only enqueues work and reads a status word.
 *
 * Operators (the problem class of the paper's experiments, section 6: viscous
 * "sinker" problems with strongly varying viscosity) are second-order finite
 * differences on the unit square/cube with homogeneous Dirichlet boundaries:
 *   (A u)_i = h^-2 sum_f k_f (u_i - u_nb) + h^-1 sum_f (max(v_f,0) u_i + min(v_f,0) u_nb)
 * over the 2*dim faces f of node i, h = 1/(n+1), u_nb = 0 on the boundary,
 * k_f = 2 eta_a eta_b / (eta_a + eta_b) (harmonic mean of the node viscosities)
 * and v_f the outward face-normal velocity (first-order upwind convection).
 * This is the 5-point (2D) / 7-point (3D) stencil of the section 7 model.
 *
 * Layouts.  Unknown vectors hold the N = n^dim interior nodes, x fastest.
 * eta holds (n+2)^dim values on the padded grid (boundary ring included), x
 * fastest.  face_vel holds three such padded arrays (x, y, z components);
 * component c at padded node p is the velocity on the face between p and
 * p + e_c.  All floating point is IEEE FP64 unless a precision option says
 * otherwise.
 *
 * Errors.  Functions return a pfk_status; a negative value is an error and
 * pfk_last_error() gives a message (per calling thread).  No exceptions cross
 * the ABI.  On any return from pfk_solve, x holds the last iterate.
 *
 * Ownership.  The caller owns b, x, the workspace and the streams it passes;
 * the library owns copies of the coefficients (made at create time), its own
 * auxiliary streams and events.  A handle may be used by one solve at a time
 * unless each concurrent solve has its own workspace and session.
 *
 * Streams.  `stream` arguments are hipStream_t values passed as void*; NULL
 * is the default stream.  Calls order themselves after work already queued on
 * that stream and leave later work on it ordered after their own.
 */
#ifndef PFK_H
#define PFK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfk_operator_s* pfk_operator;
typedef struct pfk_precond_s* pfk_precond;
typedef struct pfk_session_s* pfk_session;
typedef struct pfk_batch_s* pfk_batch;
typedef struct pfk_server_s* pfk_server;

typedef enum {
  PFK_FCG = 0,        /* Alg. 2: two blocking reductions per iteration        */
  PFK_PIPEFCG = 1,    /* Alg. 8: one reduction, overlapped with B and A        */
  PFK_GCR = 2,        /* Alg. 9                                                */
  PFK_PIPEGCR = 3,    /* Alg. 11: one reduction, overlapped with B             */
  PFK_FGMRES = 4,     /* Alg. 13                                               */
  PFK_PIPEFGMRES = 5, /* Alg. 15: one reduction, overlapped with B and A       */
  PFK_PIPEGCR_W = 6,  /* Alg. 12: PIPEGCR with w = A u recurred (a fourth window,
                         no A u per iteration), overlapped with B and A         */
  PFK_PIPEFCG_NAIVE = 7 /* Alg. 7: PIPEFCG with the unstabilised m = B(w) in place
                         of u + B(w - r); stagnates near a nonlinear B's noise
                         level (section 2.2.1).  For studying that effect.      */
} pfk_method;

typedef enum {
  PFK_PC_NONE = 0,              /* B(v) = v                                         */
  PFK_PC_JACOBI = 1,            /* B(v) = D^-1 v, D = diag(A) (linear)               */
  PFK_PC_JACOBI_PCG = 2,        /* k iterations of Jacobi-PCG on A y = v from y = 0  */
  PFK_PC_JACOBI_GMRES = 3,      /* one GMRES(k) cycle on A D^-1 t = v from 0, y = D^-1 t */
  PFK_PC_BLOCK_JACOBI_PCG = 4,  /* k Jacobi-PCG iterations inside every cubic block of
                                   `block` nodes per axis (square in 2D), on the block's
                                   principal submatrix with its own scalars: the block
                                   Jacobi of the experiments (section 6.2)             */
  PFK_PC_NOISY = 5              /* B(v) = v + eta ||v|| g/||g||, g seeded Gaussian noise:
                                   the toy of section 2.2.1; made by
                                   pfk_precond_create_noisy only                      */
} pfk_pc_kind;

typedef enum {
  PFK_FP64 = 0,            /* everything in FP64                                        */
  PFK_FP32_BF16COEF = 1    /* preconditioner inner sweeps in FP32 with BF16-stored eta;
                              the outer method stays FP64                                */
} pfk_precision;

typedef enum {
  PFK_OK = 0,
  PFK_NOT_CONVERGED = 1,   /* maxit reached (or restarts exhausted by residual gaps)  */
  PFK_ERR_ARG = -1,
  PFK_ERR_OOM = -2,
  PFK_ERR_HIP = -3,
  PFK_ERR_NONFINITE = -4,  /* NaN/Inf met in the residual                             */
  PFK_ERR_BREAKDOWN = -5   /* breakdown of the initial direction, or more than
                              max_restarts breakdown restarts                        */
} pfk_status;

typedef struct {
  int truncation;          /* window rule (section 5): 0 standard min(j, nu_max),
                              1 Notay max(1, j mod (nu_max+1)), 2 min(j, j mod nu_max + 1) */
  double shift_sigma;      /* PIPEFGMRES constant shift; NaN => estimated by
                              pfk_estimate_sigma (10 power steps)                    */
  int graph_iters;         /* iterations per captured graph launch (>= 1)            */
  int use_graph;           /* 1: replay hipGraphs; 0: launch kernels directly         */
  int host_sync;           /* FCG, GCR, FGMRES only (PFK_ERR_ARG otherwise): 1 copies
                              every reduction result to the host and waits for it
                              (a blocking reduction); turns graphs off               */
  int max_restarts;        /* breakdown / residual-gap restarts allowed               */
  int force_breakdown_at;  /* test hook: force a breakdown at this iteration (-1 off) */
  int persistent;          /* batches only: 1 runs each pfk_batch_step as one cooperative
                              launch whose phases are separated by grid barriers (no
                              kernel boundaries); 0 one launch per phase (default)    */
  int norm;                /* convergence measure of the CG/CR types: 0 the recurred
                              ||r_i||_2 <= rtol ||b||_2, then the true-residual check
                              (default); 1 the natural norm sqrt|gamma_i| <= rtol times
                              that of the first start-up, gamma = <u, r> (CG types) or
                              <r, A u> (CR types), the one norm these methods have
                              without an extra reduction (section 5); the iterate is
                              then confirmed in the natural norm of its true residual
                              r = b - A x, sqrt|<B(r), r>| (CG) or sqrt|<r, A B(r)>|
                              (CR), one more application of B, and restarted from
                              if above the tolerance (true_rel_resid reports the
                              2-norm).  GMRES types ignore it (they test the Givens
                              estimate of the preconditioned residual).              */
  int timestamps;          /* 1: record the device clock at every history entry (the
                              scalar kernel that logs it reads the GPU's constant-rate
                              wall clock); returned as iter_time_us (single solves,
                              sessions and batch members; the server does not keep
                              it)                                                    */
  int stall_window;        /* CG/CR types: 0 off (default); K > 0 restarts from x
                              (like a residual gap, counted with max_restarts) at an
                              iteration at least K after the (re)start whose recurred
                              ||r|| is above half of that K iterations earlier.  A
                              pipelined method with an inexact B can stall at a noise
                              floor scaling with ||A|| ||B|| (section 2.2.1); the
                              restart rebuilds its recurrences from the current x.
                              GMRES types ignore it.                                 */
  int side_delay;          /* test hook (single solves and sessions; batches ignore it):
                              before each reduction finish on the second
                              stream, a one-workgroup kernel sleeps this many rounds
                              of s_sleep 127 (about 3.4 us each; 0..10000, 0 off), so
                              a missing join between the streams would show in the
                              results.  Results are identical for every value.     */
} pfk_solve_opts;

typedef struct {
  int iterations;          /* solution updates (CG/CR) or Arnoldi columns (GMRES)    */
  int restarts;            /* breakdown and residual-gap restarts                     */
  int converged;           /* 1 if the true residual ended <= rtol * ||b||             */
  int status;              /* the pfk_status the solve returned                        */
  double true_rel_resid;   /* ||b - A x|| / ||b|| at exit (0 when b = 0)               */
  double* history;         /* caller buffer (host) or NULL: history[i] = residual
                              measure after iteration i (recurred ||r_i|| for CG/CR,
                              the Givens estimate for GMRES), history[0] = ||r_0||    */
  int history_cap;         /* entries available in history                            */
  int history_len;         /* entries written (iterations + 1, capped)                */
  double* natural_history; /* caller buffer (host, history_cap entries) or NULL: the
                              natural norm sqrt|gamma_i| of every iteration, [0] from
                              the first start-up (CG/CR types; logged in either norm
                              mode).  The server does not keep it.                   */
  int natural_len;         /* entries written (0 for GMRES types)                     */
  double* iter_time_us;    /* caller buffer (host, history_cap entries) or NULL: with
                              opts.timestamps, microseconds from history entry 0 to
                              entry i on the device clock                             */
  int iter_time_len;       /* entries written (0 without opts.timestamps)             */
} pfk_solve_info;

/* Defaults: standard truncation, sigma estimated, graph_iters 8, graphs on,
 * no host sync, 10 restarts, no forced breakdown, phased batches, 2-norm test. */
void pfk_default_opts(pfk_solve_opts* opts);

/* Operator A of dimension 2 or 3 with n[0..dim) interior nodes per axis (x, y, z;
 * n[0] == n[1] (== n[2]) is required: the mesh width is h = 1/(n+1) on every
 * axis).  eta: (n+2)^dim viscosities > 0; face_vel: NULL for the symmetric
 * diffusion operator, else 3*(n+2)^3 velocities (3D only).  The arrays are
 * host pointers (ptr_is_device = 0) or device pointers (1); they are copied.
 * Errors: PFK_ERR_ARG on bad sizes or non-positive eta, PFK_ERR_OOM, PFK_ERR_HIP. */
int pfk_operator_create(int dim, const int64_t n[3], const double* eta, const double* face_vel,
                        int ptr_is_device, pfk_operator* out);
void pfk_operator_destroy(pfk_operator A);
/* Number of unknowns N. */
int64_t pfk_operator_size(pfk_operator A);
/* y = A x for device vectors of N values (enqueued on stream, asynchronous). */
int pfk_operator_apply(pfk_operator A, const double* x, double* y, void* stream);
/* D^-1 (device, N values): the Jacobi scaling the preconditioners use. */
int pfk_operator_diag_inv(pfk_operator A, double* dinv, void* stream);

/* Preconditioner B of the given kind with `inner_its` inner iterations
 * (1..32, at most 8 for JACOBI_GMRES; ignored for NONE and JACOBI), precision
 * (FP32_BF16COEF applies to the three inner-iterative kinds), and `block` nodes
 * per axis for BLOCK_JACOBI_PCG (8; blocks start at interior index 0, the last
 * one per axis is ragged).  The handle refers to A, which must outlive it.
 * Errors: PFK_ERR_ARG (bad kind, count, precision or block), PFK_ERR_OOM,
 * PFK_ERR_HIP. */
int pfk_precond_create(pfk_operator A, pfk_pc_kind kind, int inner_its, pfk_precision prec,
                       int block, pfk_precond* out);
/* The noisy preconditioner of the stagnation study (section 2.2.1, Figure 1):
 * B(v) = v + eta ||v|| g / ||g|| (v unchanged when ||v|| = 0), with g standard
 * normal from a counter-based stream: node e of draw d is Box-Muller on
 * words 0 and 1 of Philox4x64-10 at counter (e, d, 0, 0) and key (seed, 0)
 * (u1 = (word0 >> 11) + 1, u2 = word1 >> 11, both times 2^-53;
 * g = sqrt(-2 ln u1) cos(2 pi u2)).  Inside a solve the draws are 0, 1, 2, ...
 * for the applications the method goes on to use, in its order (start-up
 * included, counting on across restarts; an application made concurrently
 * with the reduction that ends the solve by convergence does not count, and
 * reuses the next index).  PIPEFGMRES's shift estimate, when the library
 * makes it, draws 0, 1, ... of its own before the solve's count starts.
 * Standalone pfk_precond_apply calls use the handle's own count, 0, 1, 2, ...
 * FP64 only; not accepted by batches or the server.
 * Errors: PFK_ERR_ARG (eta negative or not finite, null pointers), PFK_ERR_OOM. */
int pfk_precond_create_noisy(pfk_operator A, double eta, uint64_t seed, pfk_precond* out);
void pfk_precond_destroy(pfk_precond B);
/* y = B(v) for device vectors, 16-byte aligned (synchronous w.r.t. stream
 * completion of the call). */
int pfk_precond_apply(pfk_precond B, const double* v, double* y, void* stream);

/* Launch geometry of A's kernels (performance only; results do not depend
 * on it beyond rounding).  tile_x: stencil tiles of 64 x 8 (64) or 32 x 16
 * (32) nodes; stencil_target: about this many workgroups per stencil launch
 * (the z-range is cut into chunks); vector_blocks: workgroups of the vector
 * kernels (window updates, multi-dots), which is also the number of partial
 * sums each reduction finishes.  A session or solve takes the geometry A has
 * when it is created.  Errors: PFK_ERR_ARG (tile_x not 32/64, counts outside
 * 1..16384). */
int pfk_operator_set_tiling(pfk_operator A, int tile_x, int stencil_target, int vector_blocks);
int pfk_operator_get_tiling(pfk_operator A, int* tile_x, int* stencil_blocks, int* vector_blocks);

typedef struct {
  int tile_x;               /* chosen stencil tile width                          */
  int stencil_target;       /* the stencil_target that gives the chosen geometry  */
  int stencil_blocks;       /* chosen workgroups per stencil launch               */
  int vector_blocks;        /* chosen workgroups per vector launch                */
  double ms_per_iteration;  /* best measured time of one outer iteration          */
  double ms_default;        /* the same with the geometry A had before            */
  int candidates;           /* configurations timed                               */
} pfk_tuning;

/* Autotuner: times outer iterations of `method` with B (window/restart mmax)
 * on this GPU for each candidate geometry -- tile widths 64 and 32 with
 * several z-chunkings, then vector workgroup counts from 64 up to N/512 --
 * and sets the fastest on A (pfk_operator_set_tiling).  CG/CR types are timed
 * over `reps` steady-state iterations, GMRES types over whole cycles.  Uses
 * library-allocated memory (about one solve's workspace) and synchronises
 * `stream`.  Errors: PFK_ERR_ARG, PFK_ERR_OOM, PFK_ERR_HIP. */
int pfk_operator_autotune(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int reps, void* stream,
                          pfk_tuning* out);

/* Bytes of workspace pfk_solve needs for this method, window/restart length
 * `mmax` (1..64) and iteration limit `maxit`. */
size_t pfk_workspace_bytes(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int maxit);

/* Solve A x = b.  b, x: device vectors of N values; x holds x0 on entry and
 * the last iterate on return.  Stops at the first iteration whose residual
 * measure is <= rtol * ||b||_2 and whose true residual confirms it, or after
 * maxit iterations.  mmax: window length nu_max (FCG/GCR types) or restart
 * length m (FGMRES types).  workspace: device memory of ws_bytes >=
 * pfk_workspace_bytes(...), 256-byte aligned, or NULL to let the library
 * allocate it for the call.  opts may be NULL (defaults); info may be NULL.  Returns PFK_OK,
 * PFK_NOT_CONVERGED or an error.  b == 0 returns x = 0 after 0 iterations. */
int pfk_solve(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
              double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes, void* stream,
              const pfk_solve_opts* opts, pfk_solve_info* info);

/* pfk_solve for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * solve, arguments and results as pfk_solve with these differences:
 *   - the workspace is a fixed device array inside the library, 256 MiB
 *     (268,435,456 bytes) on each GPU the library runs on, held until the
 *     process ends; a solve whose pfk_workspace_bytes(A, B, method, mmax,
 *     maxit) exceeds it is refused with PFK_ERR_ARG (PIPEFCG with mmax 30
 *     fits up to about 240,000 unknowns, FCG about 450,000);
 *   - every kernel runs on `stream` (the pipelined methods' second-stream
 *     work is ordered on it too; the arithmetic is the same), launched
 *     directly: no streams, events, graphs, host or device allocations;
 *   - opts->timestamps must be 0.
 * The call synchronises `stream` (the host reads the solve's status).  Every
 * call on one GPU uses that GPU's one array, which keeps the last call's
 * contents (the call clears what must start at zero): calls that overlap on
 * one GPU, from several threads or streams, race and must not be made. */
int pfk_solve_noalloc(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                      double rtol, int maxit, int mmax, void* stream, const pfk_solve_opts* opts,
                      pfk_solve_info* info);

/* Sessions split pfk_solve into asynchronous steps (for timing and serving):
 * create binds the buffers, start enqueues the set-up and start-up phase,
 * iterate enqueues `iters` more iterations without waiting, sync waits and
 * reports.  Iterations enqueued after the solve stopped change nothing. */
int pfk_session_create(pfk_operator A, pfk_precond B, pfk_method method, const double* b, double* x,
                       double rtol, int maxit, int mmax, void* workspace, size_t ws_bytes,
                       void* stream, const pfk_solve_opts* opts, pfk_session* out);
int pfk_session_start(pfk_session S);
int pfk_session_iterate(pfk_session S, int iters);
int pfk_session_sync(pfk_session S, pfk_solve_info* info);
void pfk_session_destroy(pfk_session S);

/* Kernel timing for roofline accounting: enqueues `iters` iterations with
 * kernels launched directly (no graph) and HIP events recorded on each
 * kernel's own stream right before and after it; waits, then reports per
 * kernel name (static strings owned by the library) the summed milliseconds
 * and launch count, for up to `cap` kernels.  Returns the number of distinct
 * kernels (may exceed cap) or a negative pfk_status. */
int pfk_session_profile(pfk_session S, int iters, int cap, const char** names, double* total_ms,
                        int* launches);

/* PIPEFGMRES shift: Rayleigh quotient of v -> A B(v) after `its` power steps
 * from the normalised ones vector (the largest eigenvalue of the
 * right-preconditioned operator, sections 4.4 and 5). */
int pfk_estimate_sigma(pfk_operator A, pfk_precond B, int its, double* sigma, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* pfk_last_error(void);

/* ---- batches --------------------------------------------------------------
 * Many independent systems solved together (no paper counterpart: the
 * experiments solve one system at a time).  Every phase of an outer iteration
 * is one launch covering all running members: each member owns a range of the
 * launch's workgroups sized by its own launch geometry (pfk_operator_set_tiling
 * or pfk_operator_autotune), so systems of different sizes advance in the same
 * launches; the PIPE methods' reduction finish runs on a second stream beside
 * the preconditioner and operator launches, as in a single solve.  Each member
 * computes exactly what a single pfk_solve with the same arguments computes.
 *
 * Methods: PIPEFCG, FCG, PIPEFGMRES (mmax = window or restart length).
 * Preconditioners: every kind but NOISY; all members of a batch share the
 * dimension, the preconditioner kind and its precision, and for the global
 * inner solves (JACOBI_PCG, JACOBI_GMRES) the number of inner steps: each of
 * their phases is one launch over all members.  The persistent form takes
 * NONE, JACOBI and BLOCK_JACOBI_PCG only.  opts as for
 * pfk_solve except host_sync (rejected); graph_iters iterations are captured
 * per graph (recaptured when members are added or removed, or when members
 * that ended hold half of the vector workgroups; until then an ended member's
 * launches return at once, its status being final).
 * Ownership: b, x and the workspace (or the library's allocation when NULL)
 * must stay valid while the member is in the batch. */
int pfk_batch_create(pfk_method method, int mmax, int capacity, void* stream, const pfk_solve_opts* opts,
                     pfk_batch* out);
void pfk_batch_destroy(pfk_batch T);
/* Admit one system (set-up and start-up are enqueued at once); *slot receives
 * its member index (0..capacity-1).  The workspace is sized by
 * pfk_workspace_bytes(A, B, method, mmax, maxit).  Errors: PFK_ERR_ARG (full,
 * unsupported preconditioner, a member of another kind), PFK_ERR_OOM. */
int pfk_batch_add(pfk_batch T, pfk_operator A, pfk_precond B, const double* b, double* x, double rtol,
                  int maxit, void* workspace, size_t ws_bytes, int* slot);
/* Enqueue `iters` outer iterations of every running member (asynchronous). */
int pfk_batch_step(pfk_batch T, int iters);
/* Synchronise, then act on every running member's state as pfk_solve's loop
 * does (true-residual check after a recurred convergence, restart at a GMRES
 * cycle end, after a breakdown or a residual gap).  Members that ended are
 * written to finished[0..cap) (*nfinished of them; their x is final once the
 * stream reaches this point); *nrunning counts the others.  NULL outputs ok. */
int pfk_batch_poll(pfk_batch T, int* finished, int cap, int* nfinished, int* nrunning);
/* A member's pfk_solve_info (synchronising); returns its final pfk_status, or
 * PFK_NOT_CONVERGED while it still runs. */
int pfk_batch_info(pfk_batch T, int slot, pfk_solve_info* info);
/* Test hook for the persistent form: the number of polls after which a
 * workgroup waiting at a grid barrier gives up and aborts the launch (default
 * about a second's worth).  An aborted launch leaves every member's state
 * undefined and makes the next pfk_batch_poll return PFK_ERR_HIP; the batch
 * should then be destroyed. */
int pfk_batch_set_barrier_limit(pfk_batch T, long long polls);
/* Release a member (its slot becomes free; its x keeps the last iterate). */
int pfk_batch_remove(pfk_batch T, int slot);
/* Workspace bytes of one member (the same as pfk_workspace_bytes). */
size_t pfk_batch_workspace_bytes(pfk_operator A, pfk_precond B, pfk_method method, int mmax, int maxit);
/* Solve `count` systems as one batch until every one has ended; infos[i] (may
 * be NULL) receives each system's info.  workspace: NULL (the library allocates)
 * or one device buffer holding every member's workspace in order, each
 * pfk_workspace_bytes(A[i], B[i], method, mmax, maxit) rounded up to 256 bytes.
 * Returns PFK_OK if all converged, else the first error or PFK_NOT_CONVERGED. */
int pfk_solve_batched(int count, const pfk_operator* A, const pfk_precond* B, pfk_method method,
                      const double* const* b, double* const* x, const double* rtol, int maxit, int mmax,
                      void* workspace, size_t ws_bytes, void* stream, const pfk_solve_opts* opts,
                      pfk_solve_info* infos);

/* ---- serving -------------------------------------------------------------
 * A request queue in front of continuously refilled batches (no paper
 * counterpart).  Requests are admitted in arrival order while one fits a
 * batch slot and the device-memory budget (each holds its workspace,
 * pfk_workspace_bytes, from admission to retirement; workspaces come from a
 * pool that keeps freed blocks).  Requests of one method, preconditioner kind,
 * precision and dimension share a batch; batches run on their own streams and
 * are stepped without waiting for each other, so a PIPEFCG batch and a
 * PIPEFGMRES batch overlap on the device.  A request's result is
 * bit-identical to a single pfk_solve of it, whatever else is being served.
 * Streams: admission orders a request's work after what the server's stream
 * (the `stream` of pfk_server_create) holds at that moment; the server's
 * stream is not made to wait for the batches -- a request's x is final when
 * pfk_server_progress reports it (that call synchronises the batch streams). */
typedef struct {
  size_t hbm_budget;   /* bytes of workspace the admitted requests may hold       */
  int max_active;      /* members per batch (1..4096)                             */
  int step_iters;      /* outer iterations per scheduling round (graph length)    */
  int mmax;            /* window / restart length of every request                */
  int launch_direct;   /* 1: batches launch their kernels directly instead of
                          replaying captured graphs (same results; for tools that
                          trace individual launches); 0: graphs (default)        */
  int stall_window;    /* the requests' pfk_solve_opts.stall_window (0 off)       */
  int max_restarts;    /* the requests' pfk_solve_opts.max_restarts (0: default)  */
} pfk_server_config;

typedef struct {
  long long queued, active, completed;
  size_t bytes_in_use;  /* workspaces of admitted requests                         */
  size_t bytes_held;    /* device memory the pool holds (in use or cached)         */
} pfk_server_status;

int pfk_server_create(const pfk_server_config* cfg, void* stream, pfk_server* out);
/* Destroys the batches and releases the pool (requests still running stop). */
void pfk_server_destroy(pfk_server S);
/* Queue a request; *id identifies it.  A, B, b and x stay owned by the caller
 * and must stay valid until the request has completed.  Errors: PFK_ERR_ARG
 * (method or preconditioner not batched, a request larger than the budget). */
int pfk_server_submit(pfk_server S, pfk_operator A, pfk_precond B, pfk_method method, const double* b,
                      double* x, double rtol, int maxit, long long* id);
/* One scheduling pass (admit, advance every batch by step_iters iterations,
 * poll, retire); the ids that completed in this call go to
 * completed[0..cap) (*ncompleted of them).  Synchronises the batch streams. */
int pfk_server_progress(pfk_server S, long long* completed, int cap, int* ncompleted);
/* Info of a completed request (history copied into info->history up to
 * info->history_cap); returns its final pfk_status. */
int pfk_server_result(pfk_server S, long long id, pfk_solve_info* info);
int pfk_server_stats(pfk_server S, pfk_server_status* stats);

#ifdef __cplusplus
}
#endif

#endif /* PFK_H */
