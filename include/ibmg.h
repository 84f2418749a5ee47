/*
 * ibmg.h -- C ABI of the MI355X (gfx950) implicit immersed-boundary
 * multigrid library.
 *
 * The library advances the implicit-time immersed boundary method of
 * Guy, Philip and Griffith, "Geometric multigrid for an implicit-time
 * immersed boundary method" (arXiv 1311.5614): at each time step it solves
 * the coupled Stokes-structure system (Sec. 2.3.2, eliminated to the
 * Eulerian saddle system of Sec. 3) with FGMRES right-preconditioned by the
 * geometric multigrid V-cycle of Algorithm 1 (Sec. 3), hybrid coarse
 * operators (Sec. 3.2) and (big-)box relaxation (Sec. 5-6), then moves the
 * structure with the lagged interpolation operator.
 *
 * Problem (periodic unit square, N x N cells, h = 1/N, MAC layout):
 *   (rho/dt) u - mu Lap_h u + G p + M_0 u = (rho/dt) u^n + S_0 (K L X^n) + g
 *   -D u = 0,   M_0 = -dt K S_0 L S^*,   X^{n+1} = X^n + dt S^* u^{n+1}
 * with S_0 spreading through the 4-point regularised delta (Sec. 2.2),
 * S^* = h^2 S_0^T its adjoint, L the closed-fibre second difference
 * (nodal springs, force G = K L X).  This is the unsteady form the paper
 * gives in its discussion (operator I - dt Lap - dt^2 gamma S A_f S^*,
 * Sec. 8), divided by dt.
 *
 * Memory and ownership
 *   - Every array argument is DEVICE memory owned by the caller, FP64 unless
 *     stated, except fiber_offsets (host).
 *   - Eulerian fields are N x N row-major, x fastest: u[j][i] at
 *     (i h, (j+1/2) h), v[j][i] at ((i+1/2) h, j h), p[j][i] at the cell
 *     centre.  A stacked vector w = [u; v; p] has 3 N_l^2 entries on level l
 *     (N_l = N / 2^l).
 *   - Lagrangian positions X are M x 2 (x, y interleaved), not wrapped; the
 *     kernels wrap them internally.
 *   - The library never allocates device memory: the caller queries
 *     ibmg_workspace_bytes() and binds one device buffer it owns with
 *     ibmg_bind_workspace().  The handle keeps host-side bookkeeping and a
 *     few bytes of pinned host memory.
 *   - All work is enqueued on the stream given at creation (a hipStream_t
 *     passed as void*; NULL = default stream).  Calls that return stats, or
 *     that read device scalars for control flow (solve, step, setup),
 *     synchronise that stream before returning.
 *   - One handle per host thread; handles are independent.
 *
 * Errors: every call returns an ibmg_status.  Negative values are errors;
 * on an error the caller's output buffers are left untouched (results are
 * formed in the workspace and copied out last).  IBMG_NOT_CONVERGED (> 0)
 * is a warning: outputs hold the best iterate.
 */
#ifndef IBMG_H
#define IBMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibmg_handle ibmg_handle;

typedef enum {
  IBMG_OK = 0,
  IBMG_NOT_CONVERGED = 1,   /* iteration cap reached; outputs hold the last iterate */
  IBMG_EINVAL = -1,         /* null pointer, bad enum, bad size                    */
  IBMG_ESHAPE = -2,         /* N not a power of two, box does not tile a level     */
  IBMG_EHIP = -3,           /* a HIP runtime call failed                           */
  IBMG_ENOMEM = -4,         /* bound workspace too small / not bound               */
  IBMG_ENONFINITE = -5,     /* NaN or Inf met in the inputs or the iteration       */
  IBMG_ESTATE = -6          /* call order violated (e.g. solve before setup)       */
} ibmg_status;

enum { IBMG_DELTA_IB4 = 0,  /* Peskin's standard 4-point kernel                    */
       IBMG_DELTA_COS4 = 1  /* cosine 4-point kernel printed in Sec. 2.2           */ };
enum { IBMG_FP64 = 0, IBMG_FP32 = 1 };
enum { IBMG_PERIODIC = 0, IBMG_CAVITY = 1 };
enum { IBMG_GUESS_ZERO = 0, IBMG_GUESS_PREV = 1 };
enum { IBMG_IMPLICIT = 0, IBMG_EXPLICIT = 1 };
enum { IBMG_SOLVER_FGMRES = 0, IBMG_SOLVER_MG = 1 };
enum { IBMG_ORTH_CGS2 = 0, IBMG_ORTH_DCGS2 = 1 };

typedef struct {
  int32_t N;                     /* cells per side, power of two >= 4               */
  double rho, mu;                /* density and viscosity, rho > 0, mu > 0          */
  int32_t n_points;              /* M, total Lagrangian points (may be 0)           */
  int32_t n_fibers;              /* closed fibres                                   */
  const int32_t* fiber_offsets;  /* HOST, n_fibers + 1 CSR offsets into [0, M]      */
  double K;                      /* nodal spring stiffness, force G = K L X         */
  int32_t delta;                 /* IBMG_DELTA_IB4 or IBMG_DELTA_COS4               */
  int32_t domain;                /* IBMG_PERIODIC (rho > 0) or IBMG_CAVITY: the unit
                                    square with walls on all four sides (Sec. 4), the
                                    velocity zero on them except the tangential
                                    velocity (1 - cos 2 pi x) / 2 of the top wall;
                                    rho >= 0 (0: the steady form).  Layout as
                                    periodic: the faces u[j][0] and v[0][i] lie on
                                    the walls (standing for x = 1 and y = 1 too),
                                    carry zero and are identity rows of the system;
                                    a face next to a wall parallel to it sees the
                                    ghost 2 g - u across it.  Needs opts.tail_max = 1
                                    (every smoothed level as grid-wide launches);
                                    batches take IBMG_PERIODIC only.               */
} ibmg_problem;

typedef struct {
  int32_t levels;      /* multigrid levels, coarsest N / 2^(levels-1) >= 2          */
  int32_t box;         /* box edge n in cells: 1, 2, 4 or 8; every smoothed level needs
                          N_l >= max(4, 2n) (colour classes of boxes stay disjoint)  */
  int32_t nu1, nu2;    /* pre- and post-smoothing sweeps (Algorithm 1)              */
  int32_t maxit;       /* FGMRES iteration cap over all cycles: 1..1000 when restart
                          is 0, 1..1000000 otherwise                                */
  double rtol;         /* stop when ||b - A w||_2 <= rtol ||b||_2                   */
  int32_t vcycle_prec; /* IBMG_FP64 or IBMG_FP32 (V-cycle fields and stencils)      */
  int32_t guess;       /* IBMG_GUESS_ZERO or IBMG_GUESS_PREV (step only)            */
  int32_t colours;     /* box order of a sweep: 2 = checkerboard (bx + by) mod 2,
                          4 = (bx mod 2, by mod 2) in the order (0,0),(1,0),(0,1),(1,1);
                          within a colour every box solves from the residual at
                          the start of that colour                                  */
  int32_t tail_max;    /* V-cycle schedule: levels of at most tail_max cells per
                          side (and the coarsest) run in one LDS-resident
                          workgroup, larger ones as grid-wide launches; 0 = 32,
                          else a power of two 1..32 (1: only the coarsest solve,
                          then as a grid-wide matrix-vector product).  Changes
                          the launch schedule and the summation order of the
                          elastic rows, not the method.                         */
  int32_t restart;     /* FGMRES(m) restart length m, the Krylov basis size
                          (Sec. 3.3 leaves it open): 0 = no restart below maxit
                          (m = maxit), else 1..1000 (the workspace holds 2m + 1
                          vectors of 3 N^2 doubles).  A cycle that ends without
                          meeting rtol updates the iterate and starts the next
                          cycle from its true residual.                         */
  int32_t colours_from;/* 0: every smoothed level uses `colours`; k >= 1: levels
                          k and coarser use the checkerboard (2 colours), the
                          finer ones `colours` (the order may differ per level) */
  int32_t scheme;      /* IBMG_IMPLICIT (the method: the elasticity operator in
                          the system) or IBMG_EXPLICIT (Sec. 2.3.1: the force at
                          X^n on the right-hand side only, the system is the
                          Stokes operator; stable below the explicit limit of
                          Sec. 4.1, the comparison of Sec. 7)                   */
  int32_t solver;      /* IBMG_SOLVER_FGMRES (multigrid-preconditioned FGMRES,
                          Sec. 3.3) or IBMG_SOLVER_MG (multigrid alone, Sec. 5.1:
                          w <- w + MGV(0, b - A w) until the same rtol or
                          maxit V-cycles; stats.iters counts V-cycles)          */
  double omega;        /* weight of each box correction, w[box] += omega z_box:
                          0 or 1 = the paper's undamped boxes, else (0, 1]     */
  int32_t orth;        /* FGMRES orthogonalisation (the paper fixes none):
                          IBMG_ORTH_CGS2, classical Gram-Schmidt twice (four
                          passes over the basis per iteration), or
                          IBMG_ORTH_DCGS2, the same two projections with the
                          second delayed by one iteration (one pass for the
                          products, one for the update): the same basis in
                          exact arithmetic.  The stopping test of an iteration
                          then uses its column before the delayed projection;
                          the column is completed before the iterate is
                          formed.  Batches take IBMG_ORTH_CGS2 only.        */
} ibmg_opts;

typedef struct {
  int32_t iters;          /* preconditioner applications                          */
  int32_t converged;      /* 1 if the true residual met rtol                      */
  int32_t fallback;       /* 1 if an FP32 V-cycle stalled (Arnoldi estimate down
                             by less than 10% over 20 iterations) and the solve
                             went on with the FP64 V-cycle (FGMRES is flexible:
                             the preconditioner may change between iterations) */
  int32_t guess_rejected; /* ibmg_step_x0: 1 if the proposal was dropped
                             (alpha = 0) and the solve started from w^n          */
  double rel_resid_est;   /* Arnoldi estimate |g_{j+1}| / ||b||                   */
  double rel_resid_true;  /* ||b - A w|| / ||b|| of the returned iterate          */
  double bnorm;           /* ||b||_2                                              */
  double t_setup_ms, t_solve_ms, t_step_ms;  /* host wall clock around the phases */
  double guess_alpha;     /* ibmg_step_x0: the weight alpha of the proposal      */
} ibmg_stats;

/* Create a handle.  Validates shapes (box tiling, power-of-two N, levels) and
 * stores the fibre topology.  No device work, no allocation on the device.
 * Errors: EINVAL, ESHAPE. */
int ibmg_create(ibmg_handle** out, const ibmg_problem* prob, const ibmg_opts* opts,
                void* hip_stream);
/* Bytes of device workspace the handle needs (256-byte aligned pointer). */
int ibmg_workspace_bytes(const ibmg_handle* h, size_t* bytes);
/* Bind caller-owned device memory (>= ibmg_workspace_bytes).  The first bind
 * also allocates 64 bytes of pinned host memory (freed by ibmg_destroy) that
 * the solver's per-iteration convergence flags are written into.
 * Errors: ENOMEM, EHIP. */
int ibmg_bind_workspace(ibmg_handle* h, void* dev_ptr, size_t bytes);
int ibmg_destroy(ibmg_handle* h);
const char* ibmg_status_string(int status);
/* Kernel timing of the box-relaxation phase kernel with HIP events on the
 * handle's stream (1 = on).  ibmg_phase_timing reads the accumulated total
 * (ms), the number of launches timed and their algorithmic bytes. */
int ibmg_set_timing(ibmg_handle* h, int on);
/* Kernel timing of the box-relaxation kernel alone: `reps` back-to-back
 * launches of colour `colour` on level `level` (in place on the level's
 * V-cycle iterate, in the handle's V-cycle precision), captured as a graph
 * and replayed (after one warm-up replay) between two HIP events on the
 * handle's stream.  avg_us: mean duration per launch; bytes: the
 * launch's algorithmic bytes (read residual and iterate, write iterate, per
 * unknown of the colour's boxes; the shared inverse once; each FP64 inverse
 * of a box with elastic rows once).  Needs a setup.  Synchronises. */
int ibmg_box_bench(ibmg_handle* h, int level, int colour, int reps, double* avg_us, double* bytes);
int ibmg_phase_timing(ibmg_handle* h, double* total_ms, int64_t* launches, double* bytes);
/* Kernel timing of one hot-path kernel on the current setup, `reps` launches
 * replayed from a captured graph between two HIP events on the handle's
 * stream (as ibmg_box_bench).  kernel / level / arg:
 *   IBMG_KERNEL_BOX       box relaxation on `level`, colour `arg` (= ibmg_box_bench);
 *   IBMG_KERNEL_RES       the colour phase's residual pass on `level` (Stokes
 *                         rows of every unknown and the elastic rows);
 *   IBMG_KERNEL_MULTIDOT  one classical Gram-Schmidt dot pass of FGMRES: the
 *                         first `arg` basis vectors against basis vector `arg`;
 *   IBMG_KERNEL_UPDATE    one Gram-Schmidt update pass with `arg` vectors;
 *   IBMG_KERNEL_DOT2      the delayed form's product pass: basis vectors
 *                         0 .. arg against vectors arg and arg + 1;
 *   IBMG_KERNEL_UPDATE2   the delayed form's update pass over `arg` vectors
 *                         (completes vector arg, projects vector arg + 1),
 *                         timed on zero coefficients so the basis is unchanged.
 * The Krylov kernels run on the basis left by the last solve (1 <= arg <= the
 * restart length, arg + 1 <= it for the delayed form's; results are not used).  avg_us: mean time per launch;
 * bytes: the launch's algorithmic bytes.  Needs a setup.  Synchronises. */
enum { IBMG_KERNEL_BOX = 0, IBMG_KERNEL_RES = 1, IBMG_KERNEL_MULTIDOT = 2, IBMG_KERNEL_UPDATE = 3,
       IBMG_KERNEL_DOT2 = 4, IBMG_KERNEL_UPDATE2 = 5 };
int ibmg_kernel_bench(ibmg_handle* h, int kernel, int level, int arg, int reps, double* avg_us, double* bytes);

/* Operator setup at positions X (Sec. 2.3.2 lags S at X^n; Sec. 3.2 builds the
 * coarse elasticity operators by Galerkin products; Sec. 8 notes the box
 * factors are re-formed near the structure each step): fibre forces, delta
 * weights, point-to-box binning, the elastic rows of M_0 as coefficient
 * windows and M_{l+1} = R M_l P as windows on every coarser level, box
 * inverses and the bordered coarsest inverse, for time step dt.
 * X: M x 2.  Synchronises.  Errors: EINVAL, ENOMEM, EHIP, ENONFINITE, and
 * ESHAPE when an elastic coupling reaches beyond the coefficient window
 * (fibre neighbours more than about one cell apart); the handle stays
 * usable for a setup at other positions. */
int ibmg_setup(ibmg_handle* h, double dt, const double* X);

/* One implicit IB time step (Sec. 2.3.2): setup at X^n, right-hand side,
 * FGMRES solve, zero-mean pressure, X^{n+1} = X^n + dt S^{n*} u^{n+1}.
 * u, v, p: N x N in = state n (p only used as part of the initial guess when
 * guess = PREV), out = state n+1.  X: M x 2 in/out.  g_u, g_v: body force on
 * u and v faces, nullable.  out: host stats, nullable. */
int ibmg_step(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X,
              const double* g_u, const double* g_v, ibmg_stats* out);

/* ibmg_step with a proposed initial iterate x0 (3 N^2, device, e.g. w^n plus
 * the learned correction below).  Guard: FGMRES starts from
 * w^n + alpha (x0 - w^n) with alpha = <r, q> / <q, q>, r = b - A w^n,
 * q = A (x0 - w^n), the weight that minimises ||b - A x|| on that line, so the
 * start is never worse than w^n (alpha = 0, stats.guess_rejected = 1, when q
 * vanishes or r and q are orthogonal); it then runs to the same rtol.  Errors
 * as ibmg_step. */
int ibmg_step_x0(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X,
                 const double* g_u, const double* g_v, const double* x0, ibmg_stats* out);

/* Right-hand side of the step system at the current setup (Sec. 2.3.2 with
 * the stiffness factor restored): b = [(rho/dt) u + S_0 G + g_u;
 * (rho/dt) v + S_0 G + g_v; 0].  b: 3 N^2. */
int ibmg_rhs(ibmg_handle* h, const double* u, const double* v, const double* g_u,
             const double* g_v, double* b);

/* Solve A w = b with the operator of the current setup (Sec. 3.3, FGMRES with
 * the multigrid right preconditioner).  w: 3 N^2, in = initial guess x0,
 * out = solution.  b: 3 N^2. */
int ibmg_solve(ibmg_handle* h, const double* b, double* w, ibmg_stats* out);

/* --- single operations, exported for parity checks (same kernels as the
 *     solve uses, FP64 arguments; on an FP32 handle they run the FP32
 *     kernels with conversion at entry and exit).  All need a setup. --- */
/* y = A_l w on level l (Sec. 3 matrix; level > 0 uses the hybrid operator of Sec. 3.2). */
int ibmg_apply(ibmg_handle* h, int level, const double* w, double* y);
/* r = b - A_l w. */
int ibmg_residual(ibmg_handle* h, int level, const double* b, const double* w, double* r);
/* `sweeps` box-relaxation sweeps on level l (Sec. 5-6) in place on w, in the
 * handle's colour order, each colour from the residual at its start. */
int ibmg_smooth(ibmg_handle* h, int level, const double* b, double* w, int sweeps);
/* coarse = I_{2h<-h} fine, level l -> l+1 (Sec. 3.1: R_u, R_v, R_p). */
int ibmg_restrict(ibmg_handle* h, int level, const double* fine, double* coarse);
/* fine += I_{h<-2h} coarse, level l+1 -> l (Sec. 3.1: bilinear, constant). */
int ibmg_prolong_add(ibmg_handle* h, int level, const double* coarse, double* fine);
/* Exact coarsest solve, bordered with zero-mean pressure (Algorithm 1). */
int ibmg_coarse_solve(ibmg_handle* h, const double* b, double* w);
/* z = MGV(0, r) on level 0 (Algorithm 1 with nu1, nu2 of the handle). */
int ibmg_vcycle(ibmg_handle* h, const double* r, double* z);
/* Dense box matrix A_l[box, box] (elasticity included) of box (bx, by) on
 * level l as assembled for factorisation; out: ndof x ndof row-major,
 * ndof = 2n(n+1) + n^2, local order u faces, v faces, pressures, x fastest. */
int ibmg_box_matrix(ibmg_handle* h, int level, int bx, int by, double* out);

/* --- Lagrangian-Eulerian coupling at arbitrary positions (Sec. 2.2).  These
 *     rebuild the finest-level point data for X and invalidate the setup. --- */
/* G = K L X (closed fibres).  G: M x 2. */
int ibmg_fiber_force(ibmg_handle* h, const double* X, double* G);
/* f = S_0 G on u and v faces (deterministic gather over binned points). */
int ibmg_spread(ibmg_handle* h, const double* X, const double* G, double* f_u, double* f_v);
/* U = S^* (u, v) = h^2 S_0^T (u, v).  U: M x 2. */
int ibmg_interp(ibmg_handle* h, const double* X, const double* u, const double* v, double* U);

/* ibmg_spread without a handle and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  f_u, f_v (N x N each) = S_0 G for
 * points X (M x 2) with forces G (M x 2), same kernels and bit-identical
 * results as ibmg_spread (delta kernel `delta`).  Scratch memory is a 16 MiB
 * array in device memory that each GPU holds for the life of the process,
 * shared by every call on that GPU: calls that overlap on one GPU (several
 * streams or threads) race.  Enqueued on `stream` (hipStream_t, NULL =
 * default), not synchronised.  Limits: N a power of two, 16 <= N <= 512;
 * 0 <= M <= 8192.  Errors: EINVAL (sizes beyond these limits, null pointers,
 * bad delta), EHIP. */
int ibmg_spread_noalloc(int32_t N, int32_t delta, int32_t M, const double* X, const double* G, double* f_u,
                        double* f_v, void* stream);

/* --- Batched form: many independent problems, each with its own grid,
 *     structure, stiffness, dt and options, advanced together.  Every
 *     problem runs the same method as ibmg_step (Sec. 2.3.2 step, FGMRES of
 *     Sec. 3.3, V-cycle of Algorithm 1), and its outputs are bitwise equal to
 *     ibmg_step on a handle created with the same problem and options.  The
 *     FGMRES iterations of all problems run in lockstep rounds: one launch
 *     per V-cycle step and per Krylov step covers every problem taking part,
 *     and the V-cycle over all problems is one captured graph. --- */
typedef struct ibmg_batch ibmg_batch;
/* nprob problems (1..4096); probs and opts are HOST arrays of nprob entries
 * (copied).  All opts must share vcycle_prec and take IBMG_ORTH_CGS2, all
 * problems IBMG_PERIODIC.
 * Errors as ibmg_create. */
int ibmg_batch_create(ibmg_batch** out, int32_t nprob, const ibmg_problem* probs,
                      const ibmg_opts* opts, void* hip_stream);
/* One device workspace for every problem plus the batch's tables. */
int ibmg_batch_workspace_bytes(const ibmg_batch* b, size_t* bytes);
/* Bind it (>= ibmg_batch_workspace_bytes).  Also allocates two small pinned
 * host buffers for the per-round tables.  Errors: ENOMEM, EHIP. */
int ibmg_batch_bind_workspace(ibmg_batch* b, void* dev_ptr, size_t bytes);
/* One implicit step of every problem.  dt: HOST [nprob].  u, v, p, X: HOST
 * arrays of nprob DEVICE pointers, in/out as for ibmg_step (X may be NULL
 * for a problem without points).  g_u, g_v: NULL, or HOST arrays of nprob
 * nullable DEVICE pointers.  out: HOST [nprob] stats, nullable.  Returns the
 * first error met, else IBMG_NOT_CONVERGED if any problem missed rtol, else
 * IBMG_OK.  Synchronises. */
int ibmg_batch_step(ibmg_batch* b, const double* dt, double* const* u, double* const* v,
                    double* const* p, double* const* X, const double* const* g_u,
                    const double* const* g_v, ibmg_stats* out);
/* 1 (default) = replay the captured V-cycle graph, 0 = launch it eagerly. */
int ibmg_batch_set_graph(ibmg_batch* b, int on);
/* Lockstep FGMRES rounds run so far (one host synchronisation each). */
int ibmg_batch_rounds(const ibmg_batch* b, int64_t* rounds);
int ibmg_batch_destroy(ibmg_batch* b);

/* --- Learned initial iterate (Sec. 3.3 leaves the FGMRES initial iterate
 *     free): a network Dw = F(u^n, v^n, p^n, f_u, f_v) with f = S_0 G^n the
 *     spread elastic force, proposing x0 = w^n + Dw for ibmg_step_x0.  Six
 *     3x3 periodic convolutions 5 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3 with
 *     ReLU between layers (39331 parameters, flat FP32 in layer order: W
 *     [co][ci][ky][kx] row-major, then b [co]); inputs divided by per-channel
 *     scales s_in, outputs multiplied by s_out.  BF16 weights and
 *     activations, FP32 accumulation (MFMA), FP32 masters and Adam
 *     (beta1 0.9, beta2 0.999, eps 1e-8).  Loss: mean squared error of the
 *     scaled output against (w^{n+1} - w^n) / s_out.  Planes (in5, dw3) are
 *     DEVICE FP64, stacked channel after channel, N x N each. --- */
typedef struct ibmg_cnn ibmg_cnn;
/* N: power of two, 16..4096; max_pairs: capacity of the training store
 * (a ring: the last max_pairs recorded pairs).  Errors: EINVAL, ESHAPE. */
int ibmg_cnn_create(ibmg_cnn** out, int32_t N, int32_t max_pairs, void* hip_stream);
int ibmg_cnn_workspace_bytes(const ibmg_cnn* c, size_t* bytes);
/* Bind device memory; zeroes parameters and state. */
int ibmg_cnn_bind_workspace(ibmg_cnn* c, void* dev_ptr, size_t bytes);
/* Parameters (HOST FP32 [39331]); setting them resets the Adam state. */
int ibmg_cnn_set_params(ibmg_cnn* c, const float* params);
int ibmg_cnn_get_params(ibmg_cnn* c, float* params);
/* Scales (HOST FP32: s_in[5], s_out[3], all > 0).  Unset, the first
 * ibmg_cnn_train sets each to the RMS of its channel over the stored pairs
 * (1 for an all-zero channel).  get: s8 = s_in then s_out.  */
int ibmg_cnn_set_scales(ibmg_cnn* c, const float* s_in5, const float* s_out3);
int ibmg_cnn_get_scales(ibmg_cnn* c, float* s8);
/* Store one training pair (input planes in5 [5 N^2], target dw3 [3 N^2]). */
int ibmg_cnn_record(ibmg_cnn* c, const double* in5, const double* dw3);
int ibmg_cnn_pairs(const ibmg_cnn* c, int32_t* n);
/* `epochs` passes over the stored pairs in recording order, one Adam step
 * per pair at learning rate lr; mean loss of the first and last epoch
 * (HOST, nullable).  Synchronises.  Errors: ESTATE (no pairs). */
int ibmg_cnn_train(ibmg_cnn* c, int32_t epochs, float lr, float* loss_first, float* loss_last);
/* dw3 = F(in5) (device).  Errors: ESTATE (scales unset). */
int ibmg_cnn_infer(ibmg_cnn* c, const double* in5, double* dw3);
/* Loss and gradient (HOST FP32 [39331]) of one pair, no update.  Synchronises. */
int ibmg_cnn_loss_grad(ibmg_cnn* c, const double* in5, const double* dw3, float* loss, float* grad);
int ibmg_cnn_destroy(ibmg_cnn* c);

/* --- The learned initial iterate bound to the solver (Sec. 3.3 leaves the
 *     FGMRES initial iterate free).  The network handle c (same N and the
 *     same stream as the solver handle h) keeps the trajectory's previous
 *     increment dw^{n-1} = w^n - w^{n-1} (zero after binding or
 *     ibmg_guess_reset).  ibmg_guess_step is one implicit step (as ibmg_step,
 *     same arguments) whose initial iterate depends on mode:
 *       IBMG_GUESS_RECORD   from w^n; afterwards the training pair
 *                           (features of step n, dw^n - dw^{n-1}) is stored
 *                           in c (ibmg_cnn_record);
 *       IBMG_GUESS_EXTRAP   x0 = w^n + dw^{n-1} (first-order extrapolation);
 *       IBMG_GUESS_LEARNED  x0 = w^n + dw^{n-1} + F(features), F the
 *                           network (scales must be set, e.g. by training).
 *     Both proposals go through ibmg_step_x0's guard (the minimal-residual
 *     point on the line from w^n through x0), and the solve runs to rtol as
 *     always.  Features: (u^n, v^n, p^n, S_0 G^n on u faces, on v faces),
 *     formed on the device from the step's setup.  Every mode updates
 *     dw^{n-1}.  Synchronises.  Errors: as ibmg_step; EINVAL for a network of
 *     another size or stream, ESTATE (learned) when the scales are unset. --- */
enum { IBMG_GUESS_RECORD = 0, IBMG_GUESS_EXTRAP = 1, IBMG_GUESS_LEARNED = 2 };
int ibmg_guess_step(ibmg_handle* h, ibmg_cnn* c, int mode, double dt, double* u, double* v, double* p, double* X,
                    const double* g_u, const double* g_v, ibmg_stats* out);
/* Forget the previous increment (the next step starts a trajectory). */
int ibmg_guess_reset(ibmg_cnn* c);
/* Copy the previous increment dw^{n-1} (3 N^2, device) out of / into the
 * network handle, e.g. to run several forms of a trajectory from one state. */
int ibmg_guess_get_increment(ibmg_cnn* c, double* dw3);
int ibmg_guess_set_increment(ibmg_cnn* c, const double* dw3);

#ifdef __cplusplus
}
#endif
#endif /* IBMG_H */
