/*
 * stp.h -- C-ABI of the space-time parabolic solver for MI355X (gfx950).
 *
 * The library solves the space-time discretisation of the heat equation
 *     du/dt - Laplace(u) = g  on (0,1)^2 x (0,1),  u = 0 on the boundary,  u(0) = u0
 * by the method of van Venetie & Westerdiep, "A parallel algorithm for solving
 * linear parabolic evolution equations" (arXiv 2009.08875):
 *   - trial space: continuous piecewise linears in time (N = 2^J uniform
 *     intervals) times P1 finite elements on the uniform 2^K x 2^K square mesh
 *     cut along its "/" diagonals (Section 4, Section 5.1);
 *   - the Schur-complement system S u = f of eq. (8), written as in Lemma 4.2
 *     with K_x = two symmetric multigrid V-cycles for A_x (Section 3.1, 5.1);
 *   - PCG on the wavelet-in-time system S-hat w = f-hat, S-hat = W^T S W, with
 *     the block-diagonal preconditioner K_X of Theorem 3.1 (alpha = 0.3), and
 *     u = W w (Section 3.3, Section 3.4).
 *
 * Conventions (every entry point):
 *   - Arrays are FP64, time-major: a space-time array holds (2^J + 1) rows of
 *     N_x = (2^K - 1)^2 values; row i is the nodal vector at t_i = i / 2^J, and
 *     node (x_a, y_b) = (a h, b h), 1 <= a, b <= 2^K - 1, h = 2^-K, sits at
 *     offset (b - 1)(2^K - 1) + (a - 1).  Boundary values are zero and omitted.
 *   - on_device = 0: the pointer is host memory; it is read or written before
 *     the call returns.  on_device = 1: the pointer is device memory on the
 *     context's device; it is read or written in order on the context's stream,
 *     so the caller keeps it alive until that stream has been synchronised.
 *   - The caller owns every buffer it passes; the library owns every device
 *     allocation made inside a context or server.
 *   - Every function returns stp_status (0 = STP_OK) and never throws.  A
 *     positive status is a warning; a negative one an error.  stp_last_error()
 *     gives a readable description of the calling thread's last failure.
 *     After STP_E_DEVICE the context must be destroyed.
 */
#ifndef STP_H
#define STP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int stp_status;
#define STP_OK                 0
#define STP_NOT_CONVERGED      1   /* maxit reached; the iterate is readable */
#define STP_E_INVALID_ARG     -1   /* argument out of range, NULL where required, wrong state */
#define STP_E_OUT_OF_MEMORY   -2   /* device allocation failed or budget exceeded */
#define STP_E_BREAKDOWN       -3   /* PCG breakdown: p^T S-hat p <= 0 or a non-finite scalar */
#define STP_E_DEVICE          -4   /* a HIP call failed; the context is unusable */
#define STP_E_UNSUPPORTED     -5   /* valid request this build does not handle */
#define STP_E_BUSY            -6   /* server: result not ready yet */

typedef enum {
  STP_FP64 = 0,   /* FP64 storage and arithmetic throughout */
  STP_MIXED = 1   /* FP32 inner PCG (storage and arithmetic of every operator),
                     FP64 dot products and scalars, FP64 outer residual
                     f-hat - S-hat w and FP64 refinement w += d */
} stp_precision;

/* Options; a zero-initialised struct selects the paper's settings
 * (Section 5.1, Section 5.2): alpha = 0.3, 2 V-cycles, 3 smoothing steps. */
typedef struct {
  double alpha;      /* alpha in K_j = (alpha A_x + 2^j M_x)^{-1}; 0 -> 0.3 */
  int vcycles;       /* V-cycles per multigrid application; 0 -> 2 */
  int sweeps;        /* Gauss-Seidel steps before and after the coarse grid; 0 -> 3 */
  int maxit;         /* PCG iteration limit (inner limit in STP_MIXED); 0 -> 200 */
  double inner_tol;  /* STP_MIXED: relative reduction per inner solve; 0 -> by mesh:
                        1e-4 for K <= 7, 1e-3 for K = 8, 3e-3 for K >= 9 */
  int max_outer;     /* STP_MIXED: refinement-step limit; 0 -> 20 */
  int graph;         /* replay each PCG iteration from a captured HIP graph:
                        0 (default) or 1 -> yes (not while profiling), -1 -> no */
  int nested;        /* STP_FP64: nested iteration (Section 4.2) over up to this many
                        coarser meshes (J - d, K - d), d = 1..min(nested, J, K - 1):
                        the coarsest is solved from w = 0 to rel_tol * 2^d, every
                        finer one from the coarser solution (coarse wavelet
                        coefficients on the even time rows, P1 interpolation in
                        space) to rel_tol * 2^d, the target mesh (d = 0) to rel_tol.
                        The data of a coarser mesh are g and u0 at its nodes.  The
                        stopping test stays relative to f-hat^T K_X f-hat of each
                        mesh.  0 (default): off.  The coarser meshes are allocated
                        with the context (at most 1/7 of its memory more; not
                        counted by stp_footprint). */
  double diffusion[3];  /* the reaction-diffusion operator of Section 4,
                           a(eta, zeta) = int D grad eta . grad zeta + c eta zeta:
                           D = [[d0, d2], [d2, d1]], constant, symmetric positive
                           definite (all three 0 -> identity, the heat equation) */
  double reaction;      /* c >= 0 (0: no reaction term) */
  int dim;              /* space dimensions: 0 or 2 -> the unit square; 3 -> the unit
                           cube of Section 5.2's 3D problem on the Kuhn tetrahedral mesh
                           (each cube cut into 6 tetrahedra around its (1,1,1) diagonal),
                           1 <= K <= 8, N_x = (2^K - 1)^3, node (a, b, c) at offset
                           ((c - 1)(2^K - 1) + (b - 1))(2^K - 1) + (a - 1); the heat
                           equation only (no nesting, diffusion or reaction), not for
                           the server; stp_footprint counts two dimensions */
  int lookahead;        /* when the host reads the per-right-hand-side convergence
                           flags (Section 3.4's stopping test is taken on the device):
                           0 (default) -> after a batch of PCG iterations of half the
                           remaining count that the observed mean reduction of
                           sqrt(r^T z) per iteration predicts (all remaining ones
                           with rel_tol = 0); -1 -> after every iteration.  Iterations
                           past a right-hand side's stop change nothing of it, so
                           results and iteration counts do not depend on this */
} stp_options;

typedef struct {
  int iterations;        /* S-hat applications of the (inner) PCG, summed */
  int outer_iterations;  /* STP_MIXED: FP64 residuals r = f-hat - S-hat w evaluated,
                            counting r = f-hat of w = 0 (0 for STP_FP64) */
  double rel_residual;   /* sqrt(r^T K_X r / f-hat^T K_X f-hat) of the returned w.
                            STP_FP64: PCG's own r and z.  STP_MIXED: r is the FP64
                            residual of the returned w, rounded to FP32, and K_X the
                            FP32 preconditioner, so the value carries the FP32 K_X's
                            rounding (a relative error of a few 1e-3 at h = 2^-9) */
  double seconds;        /* device time of the solve (HIP events on the stream) */
  int status;            /* per right-hand side: STP_OK, STP_NOT_CONVERGED, STP_E_BREAKDOWN */
  int coarse_iterations; /* nested iteration: S-hat applications on the coarser meshes,
                            summed (0 without nesting) */
} stp_stats;

typedef struct stp_ctx stp_ctx;

/* Create a solver for N = 2^J time intervals (0 <= J <= 14), a 2^K x 2^K
 * mesh (1 <= K <= 10) and nrhs >= 1 independent right-hand sides sharing the
 * mesh, solved together (one launch per operator covers all of them).
 * hip_stream: a hipStream_t to run on (NULL = the library creates its own).
 * Allocates all device memory of the context; STP_E_OUT_OF_MEMORY if it does
 * not fit.  u0 and g start at zero. */
stp_status stp_create(int J, int K, int nrhs, int precision, const stp_options* opt,
                      void* hip_stream, stp_ctx** out);

/* u0: N_x values for right-hand side `rhs` (nodal interpolant, Lemma 4.1's u_0). */
stp_status stp_set_u0(stp_ctx* ctx, int rhs, const double* u0, int on_device);

/* g: (2^J + 1) x N_x nodal values of the forcing for right-hand side `rhs`;
 * NULL sets g = 0.  The data are interpolated (continuous piecewise linear in
 * time, P1 in space) and integrated exactly (Lemma 4.1's g). */
stp_status stp_set_g(stp_ctx* ctx, int rhs, const double* g, int on_device);

/* Solve every right-hand side to sqrt(r^T K_X r) <= rel_tol sqrt(f-hat^T K_X f-hat)
 * (r = f-hat - S-hat w, w_0 = 0; the quantity of eq. (13)).  rel_tol = 0
 * runs exactly maxit iterations.  per_rhs (may be NULL) receives nrhs entries.
 * Returns STP_OK, STP_NOT_CONVERGED (some rhs hit maxit), STP_E_BREAKDOWN. */
stp_status stp_solve(stp_ctx* ctx, double rel_tol, stp_stats* per_rhs);

/* u = W w of the last solve (Section 3.4: the solution of S u = f is
 * recovered from the wavelet coordinates w of S-hat w = f-hat by one
 * synthesis): (2^J + 1) x N_x nodal values, written to `u` (host or device
 * memory of the caller, layout as above).  STP_E_INVALID_ARG before the first
 * solve, for a NULL `u` or an `rhs` out of range. */
stp_status stp_get_solution(stp_ctx* ctx, int rhs, double* u, int on_device);
/* PCG iterations of the last solve of right-hand side `rhs`: the number of
 * S-hat applications (Section 3.4; in STP_MIXED the inner FP32 iterations,
 * summed over the refinement steps).  0 before the first solve;
 * STP_E_INVALID_ARG for a NULL output or an `rhs` out of range. */
stp_status stp_get_iterations(const stp_ctx* ctx, int rhs, int* iterations);

/* Device bytes held by a context with these sizes (planning / admission). */
stp_status stp_footprint(int J, int K, int nrhs, int precision, size_t* bytes);

void stp_destroy(stp_ctx* ctx);

const char* stp_status_string(stp_status s);
const char* stp_last_error(void);

/* ---- single operators, for parity checks of each step -------------------
 * stp_apply reads `in` and writes `out`, both (2^J + 1) x N_x FP64 arrays of
 * right-hand side `rhs`, using the kernels of precision `precision`
 * (STP_MIXED = the FP32 kernels: the input is rounded to FP32, the result
 * widened to FP64).  The operators are:                                     */
#define STP_OP_W       0  /* synthesis W_t (x) Id: wavelet -> nodal (Section 3.3) */
#define STP_OP_WT      1  /* analysis (W_t (x) Id)^T                              */
#define STP_OP_S       2  /* S of Lemma 4.2 (nodal)                               */
#define STP_OP_SHAT    3  /* S-hat = W^T S W (eq. (11))                    */
#define STP_OP_KX      4  /* K_X of Theorem 3.1 on wavelet coordinates           */
#define STP_OP_KSPACE  5  /* K_x (two V-cycles for A_x) on every time row         */
#define STP_OP_RHS     6  /* f of Lemma 4.1 from the context's g and u0; `in` unused */
#define STP_OP_A       7  /* A_x on every time row                                */
#define STP_OP_M       8  /* M_x on every time row                                */
stp_status stp_apply(stp_ctx* ctx, int op, int precision, int rhs,
                     const double* in, double* out, int on_device);

/* ---- kernel timing, for roofline reports ------------------------------
 * While enabled, the library brackets every launch of its hot kernels with
 * HIP events on the context stream and accumulates, per kernel, the number
 * of launches, their summed device time and their algorithmic HBM bytes
 * (each input element read once, each output element written once, over the
 * interior nodes).  Profiling runs every PCG iteration eagerly (no graph
 * replay), so time solves with it off and profile a separate solve.
 * Kernels (the steps of Section 3.4's iteration and Lemma 4.2's S):        */
#define STP_KERNEL_MG_PRE        0  /* finest-grid pre-smoothing + restriction (K_x, K_l) */
#define STP_KERNEL_MG_POST       1  /* finest-grid prolongation + post-smoothing           */
#define STP_KERNEL_SYN_UPDATE    2  /* X = W (z + beta p), p updated (eq. (11), Section 3.3) */
#define STP_KERNEL_ANA_DOT       3  /* q = W^T q with p^T q, both passes                    */
#define STP_KERNEL_TIME_STENCIL  4  /* y1, y2 of Lemma 4.2 (time and space stencils)        */
#define STP_KERNEL_COMBINE       5  /* M z1 + A z2 (+ Gamma_0 term)                          */
#define STP_KERNEL_UPDATE_WR     6  /* w += gamma p, r -= gamma q                            */
#define STP_KERNEL_DOT           7  /* r^T z, both passes                                    */
#define STP_KERNEL_COUNT         8
typedef struct {
  int launches;
  double total_ms;
  double alg_bytes;   /* summed over the launches */
} stp_kernel_stat;
stp_status stp_profile(stp_ctx* ctx, int enable);          /* enabling also clears */
stp_status stp_profile_read(stp_ctx* ctx, int kernel, stp_kernel_stat* out);

/* ---- K_x without device allocation -------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * what stp_apply(STP_OP_KSPACE) computes in FP64 -- K_x, two V-cycles from
 * zero for A_x (Section 3.1, Section 5.1), on every one of `rows` rows of
 * N_x = (2^K - 1)^2 nodal values -- without a context.
 *   in, out:   device pointers on the current device, rows x N_x FP64 values
 *              each (layout as above), owned by the caller; must not overlap.
 *   hip_stream: the hipStream_t the work is enqueued on (NULL = null stream);
 *              the call returns without waiting for it.
 * Every intermediate lives in one fixed device array of
 * STP_STATIC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends; rows are processed in chunks that fit it
 * (a row of level K takes about 32 (2^K)^2 bytes), so any `rows` works.
 * The call makes no hipMalloc, hipFree or other allocation, no trial launches
 * of the launch-shape tuner, and no wait.  All calls on one device share the
 * array: calls that overlap in time on one device race and must be ordered
 * (one stream, or events).  Errors: STP_E_INVALID_ARG (K outside [1, 10],
 * rows < 0, a NULL buffer), STP_E_DEVICE (no current device, launch failure). */
#define STP_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
stp_status stp_kspace_apply_static(int K, int rows, const double* in, double* out,
                                   void* hip_stream);

/* ---- serving: continuous batching of independent solves ------------------
 * Not in the paper (its method solves one problem at a time); this is the
 * request loop around the same solver.  A server owns a device byte budget,
 * up to four HIP streams and a worker thread on the device that is current
 * when it is created.  Requests wait in arrival order; when a slot is free and
 * the head request's context (stp_footprint) fits in the budget, the worker
 * admits it together with up to max_batch - 1 waiting requests of the same
 * (J, K, precision) whose tolerance is within a factor of 10 of its own, as
 * the right-hand sides of one batched context (groups of 1, 2, 4, ...
 * requests; only problems whose single context is at most 2 GiB are grouped:
 * a larger one fills the device alone).  Running groups advance independently, one PCG
 * iteration or refinement step at a time, on separate streams, so requests
 * admitted while others run overlap with them on the device.  Every
 * right-hand side of a group computes exactly its solo solve (its own
 * tolerance, scalars and stopping), so results do not depend on the mix.
 * A finished group writes its solutions and releases its slot at once; its
 * context is kept for a later group of the same shape and freed when the
 * budget needs the room.                                                      */
typedef struct stp_server stp_server;

typedef struct {
  int J, K;            /* sizes as in stp_create */
  int precision;       /* STP_FP64 or STP_MIXED */
  double rel_tol;      /* as in stp_solve */
  const double* u0;    /* N_x values; NULL -> u0 = 0 */
  const double* g;     /* (2^J + 1) x N_x nodal values; NULL -> g = 0 */
  double* u;           /* receives the solution, (2^J + 1) x N_x; NULL -> not kept */
  int on_device;       /* 1: u0, g and u are device pointers on the server's device */
} stp_request;
/* The buffers of a request are read when the request is admitted and u is
 * written when it finishes; the caller keeps them alive until
 * stp_server_poll reports the request finished.  The server reads device
 * buffers on its own streams, which are not ordered after any of the
 * caller's streams: the values in u0 and g must be complete (the stream or
 * event that produced them synchronised) before stp_server_submit. */

typedef struct {
  int waiting;                /* requests not yet admitted */
  int running_groups;         /* groups on the device */
  int unfinished;             /* submitted and not finished */
  size_t bytes_in_use;        /* running and cached contexts */
  size_t peak_bytes;
  int64_t groups_started;
  int64_t requests_started;   /* requests_started / groups_started = mean batch */
} stp_server_stats;

/* opt: solver options for every context (NULL = defaults).  Errors:
 * STP_E_INVALID_ARG (budget 0, max_slots or max_batch outside [1, 64]). */
stp_status stp_server_create(size_t hbm_budget_bytes, int max_slots, int max_batch,
                             const stp_options* opt, stp_server** out);
/* Queue a request; *id identifies it.  STP_E_OUT_OF_MEMORY when a single
 * request of this size cannot fit in the budget; STP_E_INVALID_ARG for bad
 * sizes.  Thread-safe. */
stp_status stp_server_submit(stp_server* s, const stp_request* req, uint64_t* id);
/* STP_E_BUSY while the request waits or runs.  Once finished: returns the
 * request's status (STP_OK, STP_NOT_CONVERGED, STP_E_BREAKDOWN or the error
 * that stopped it), fills stats and the seconds from submission to completion
 * (either may be NULL), and forgets the id.  Thread-safe. */
stp_status stp_server_poll(stp_server* s, uint64_t id, stp_stats* stats, double* latency_seconds);
/* Block until every submitted request has finished. */
stp_status stp_server_drain(stp_server* s);
stp_status stp_server_info(stp_server* s, stp_server_stats* out);
/* Finish every submitted request, then free the server and its contexts. */
stp_status stp_server_destroy(stp_server* s);

#ifdef __cplusplus
}
#endif
#endif /* STP_H */
