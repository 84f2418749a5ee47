/* Three-dimensional form of the implicit immersed-boundary multigrid solve
 * (C ABI).
 *
 * The paper states its method in two dimensions and notes that the
 * formulation, the hybrid multigrid of Sec. 3 and the big-box smoother of
 * Sec. 6 carry over to three, where a box of n^3 cells holds
 * 3 (n + 1) n^2 velocities and n^3 pressures (304 unknowns, a dense block of
 * about 750 KB, for n = 4; discussion of solver performance).  This header
 * exposes that extension on the periodic unit cube:
 *
 *   - MAC grid, N cells per side, h = 1/N: u[k][j][i] at (i h, (j+1/2) h,
 *     (k+1/2) h), v at ((i+1/2) h, j h, (k+1/2) h), w at ((i+1/2) h,
 *     (j+1/2) h, k h), p at cell centres; flat index (k N + j) N + i.  A
 *     level vector is [u; v; w; p] (4 N^3 doubles).
 *   - Level system of the implicit step (Sec. 2.3.2, unsteady operator of
 *     the discussion, divided by dt): per velocity component a,
 *     (rho/dt - mu Lap) u_a + G_a p + M_a u_a, continuity -D u, with
 *     M_a = -dt K S_a L J_a (S_a spreads with the tensor-product delta
 *     divided by h^3, J_a = h^3 S_a^T interpolates, L is the second
 *     difference along each closed fibre).
 *   - Coarse levels (Sec. 3.2): Stokes re-discretised, elasticity Galerkin
 *     M_{l+1} = R M_l P with the face transfers of Sec. 3.1 taken axis by
 *     axis (full weighting along the normal, two-point averages across; linear
 *     along the normal, 3/4-1/4 across).
 *   - Smoother (Sec. 5-6): boxes of n^3 cells (n = 2 or 4) with all faces of
 *     their cells, solved exactly, checkerboard by (bx + by + bz) mod 2,
 *     Jacobi within a colour, optional weight omega.
 *   - Coarsest level (Algorithm 1): exact solve of the system bordered by the
 *     pressure constant (zero-mean pressure).
 *   - FGMRES right-preconditioned by one V-cycle (Sec. 3.3), classical
 *     Gram-Schmidt applied twice in its delayed (low-synchronisation) form.
 *
 * Memory: every pointer argument is device memory owned by the caller; the
 * library allocates no device memory (the caller binds one workspace of
 * ibmg3_workspace_bytes()).  All work runs on the stream given at creation.
 * Status codes are those of ibmg.h.
 */
#ifndef IBMG3_H
#define IBMG3_H

#include "ibmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibmg3_handle ibmg3_handle;

typedef struct {
  int32_t N;                    /* cells per side: power of two, 8 <= N <= 128 */
  double rho, mu;               /* rho > 0, mu > 0 */
  int32_t M;                    /* Lagrangian points (0: no structure) */
  int32_t nfib;                 /* closed fibres */
  const int32_t* fiber_offsets; /* host, nfib + 1 offsets, every fibre >= 3 points */
  double K;                     /* nodal stiffness of G = K L X (>= 0) */
  int32_t delta;                /* IBMG_DELTA_IB4 or IBMG_DELTA_COS4 */
} ibmg3_problem;

typedef struct {
  int32_t levels;   /* >= 2; every smoothed level N_l has N_l / box even; coarsest N_c in 2..4 */
  int32_t box;      /* box edge n: 2 or 4 */
  int32_t nu1, nu2; /* pre- and post-smoothing sweeps, 0..8 */
  int32_t maxit;    /* FGMRES iterations (no restart), 1..500 */
  double rtol;      /* stop when ||b - A x|| <= rtol ||b|| */
  double omega;     /* box correction weight, 0 < omega <= 1 */
} ibmg3_opts;

/* Validate the problem and options, keep a host copy of the fibres.
 * Errors: EINVAL (argument out of range, a fibre under 3 points), ENOMEM. */
int ibmg3_create(ibmg3_handle** out, const ibmg3_problem* prob, const ibmg3_opts* opts, void* hip_stream);
int ibmg3_workspace_bytes(const ibmg3_handle* h, size_t* bytes);
/* Bind caller-owned device memory (>= ibmg3_workspace_bytes, 256-byte
 * aligned).  Also allocates 64 bytes of pinned host memory for the solver's
 * per-iteration flags.  Errors: ENOMEM, EHIP. */
int ibmg3_bind_workspace(ibmg3_handle* h, void* dev_ptr, size_t bytes);
int ibmg3_destroy(ibmg3_handle* h);

/* Build the hierarchy for time step dt at positions X (device, M x 3,
 * unwrapped, row-major): delta windows on every level, the elastic rows, the
 * box inverses of boxes that meet the structure (one dense 304 x 304 inverse
 * each for n = 4) and the shared inverse of the plain box, the bordered
 * coarsest inverse.  Synchronises the stream once (box lists).
 * Errors: ESTATE (no workspace), EINVAL (dt <= 0), ENONFINITE, EHIP. */
int ibmg3_setup(ibmg3_handle* h, double dt, const double* X);

/* y = A_l x on level l (4 N_l^3 each).  Errors: ESTATE (no setup), EINVAL. */
int ibmg3_apply(ibmg3_handle* h, int32_t level, const double* x, double* y);
/* rc = R rf (level -> level + 1) and wf += P ec (level + 1 -> level). */
int ibmg3_restrict(ibmg3_handle* h, int32_t level, const double* rf, double* rc);
int ibmg3_prolong_add(ibmg3_handle* h, int32_t level, const double* ec, double* wf);
/* The box block of level l's matrix for box (bx, by, bz), row-major
 * (ndof x ndof, unknowns ordered u, v, w, p, x fastest within each). */
int ibmg3_box_matrix(ibmg3_handle* h, int32_t level, int32_t bx, int32_t by, int32_t bz, double* out);
/* `sweeps` checkerboard sweeps of the box smoother on level l, w updated. */
int ibmg3_smooth(ibmg3_handle* h, int32_t level, const double* b, double* w, int32_t sweeps);
/* z = MGV(0, r) on level 0 (Algorithm 1). */
int ibmg3_vcycle(ibmg3_handle* h, const double* r, double* z);
/* b = (rho/dt) [u; v; w] + S (K L X) on the velocity rows, 0 on continuity;
 * uvw is 3 N^3 (u, v, w); X (M x 3, null without structure) must be the
 * positions of the last setup (S is that setup's spreading). */
int ibmg3_rhs(ibmg3_handle* h, const double* uvw, const double* X, double* b);
/* FGMRES on the level-0 system from the initial iterate in x (4 N^3).
 * Returns OK or NOT_CONVERGED (x holds the last iterate). */
int ibmg3_solve(ibmg3_handle* h, const double* b, double* x, ibmg_stats* st);
/* One implicit step: setup at X^n, right-hand side, solve from [uvw; p],
 * then X += dt J u.  uvw (3 N^3) and p (N^3) are updated in place. */
int ibmg3_step(ibmg3_handle* h, double dt, double* uvw, double* p, double* X, ibmg_stats* st);
/* Boxes of level l that meet the structure (own inverses) and all boxes. */
int ibmg3_box_counts(const ibmg3_handle* h, int32_t level, int32_t* own, int32_t* total);

#ifdef __cplusplus
}
#endif
#endif
