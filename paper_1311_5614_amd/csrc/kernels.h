// Launch wrappers and small utility kernels shared by the translation units.
#pragma once
#include "common.h"

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ x, size_t n, T v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void __launch_bounds__(256) static k_fill_i32(int* __restrict__ x, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <typename S, typename D>
__global__ void __launch_bounds__(256) k_convert(const S* __restrict__ a, D* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (D)a[i];
}

// The V-cycle's level-0 input in its own precision (b = r) and its initial
// iterate (w = 0), one pass.
template <typename D>
__global__ void __launch_bounds__(256) k_vcycle_in(const double* __restrict__ r, D* __restrict__ b, D* __restrict__ w,
                                                   size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    b[i] = (D)r[i];
    w[i] = D(0);
  }
}

// out = a + sb b (+ sc c when c is given), elementwise over n: the FP64
// vector sums of the learned initial iterate (proposal, increment, target).
// (out may be a or c: each lane reads its entries before it writes)
__global__ void __launch_bounds__(256) static k_lincomb(double* out, const double* a, const double* __restrict__ b,
                                                       double sb, const double* c, double sc, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = a[i] + sb * b[i];
  if (c) x += sc * c[i];
  out[i] = x;
}

struct ibmg_cnn;

namespace ibmg {

inline unsigned nblk(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }

// Trajectory state a warm-start network handle keeps for ibmg_guess_step
// (device FP64 planes of N x N): the step's features (u, v, p, then the spread
// elastic force on u and v faces, and a sixth plane the spreading pass also
// writes), w^n, the previous increment dw^{n-1}, the proposal and the new
// increment.
struct CnnTraj {
  int N = 0;
  hipStream_t stream = nullptr;
  double *feat = nullptr, *wold = nullptr, *dprev = nullptr, *x0 = nullptr, *dw = nullptr;
};
int cnn_traj(ibmg_cnn* c, CnnTraj* t);

// ib_setup.hip
void launch_fiber_force(hipStream_t s, int M, const int* prev, const int* next, double K,
                        const double* X, double* G);
void launch_weights0(hipStream_t s, int M, int N, int kind, const double* X, int* org, double* w);
void launch_scan(hipStream_t s, const int* in, int n, int* out, int* rows, int cap, int* total, int* loc,
                 int* bsum);
void launch_box_lists(hipStream_t s, const PointView& P, int* cnt, int* start, int* cursor, int* list,
                      int max_list, int* total, int* loc, int* bsum);
void launch_active(hipStream_t s, int level, int M, int N, const int* org, const int* act_fine, int* flag,
                   int* act, int* rows, int* nact, int maxact, int* loc, int* bsum);
void launch_windows0(hipStream_t s, const PointView& P, const int* rows, const int* nact, int maxact, double kappa,
                     int reach, double* win, int* flags);
void launch_windows_coarse(hipStream_t s, int Nc, const int* act_f, const double* win_f, int maxact_f, int reach_f,
                           const int* rows, const int* nact, int maxact, int reach, double* win, int* flags,
                           int walls = 0);
void launch_box_classes(hipStream_t s, int N, int n, int nb, int ncol, const int* act, int walls, int* flag,
                        int* ib_index, int* ib_boxes, int* info);
// per-colour lists of the active rows of a four-colour level (LevelView::crow)
void launch_colour_rows(hipStream_t s, int N, int n, int nb, const int* rows, const int* nact, int maxact, int* crow,
                        int* ncrow);
// Box inverses of every non-coarsest level in one launch: level l owns blocks
// first[l] .. first[l + 1] - 1, the first of them its plain block and the
// others its boxes with elastic rows (ib_boxes[l]).
struct BoxFactorLevels {
  LevelView<double> v[IBMG_MAX_LEVELS - 1];
  const int* ib_boxes[IBMG_MAX_LEVELS - 1];
  double* ainv_plain[IBMG_MAX_LEVELS - 1];
  float* ainv_plain_f[IBMG_MAX_LEVELS - 1];
  double* ainv_ib[IBMG_MAX_LEVELS - 1];
  int first[IBMG_MAX_LEVELS];
  int nl;
};
static_assert(sizeof(BoxFactorLevels) <= 4096, "kernel argument size");
void launch_box_factor(hipStream_t s, const BoxFactorLevels& F);
void launch_box_matrix(hipStream_t s, const LevelView<double>& L, int bx, int by, double* out);

// mg.hip (T = double or float)
template <typename T> void launch_residual(hipStream_t s, const LevelView<T>& L, const T* b, const T* w, T* r,
                                           bool ib);
template <typename T> void launch_res(hipStream_t s, const LevelView<T>& L, const T* b, const T* w, T* r, bool ib);
// ib: boxes listed in L.ib_index take their own inverse (boxes with elastic
// rows, and with walls the boxes touching a wall)
template <typename T> void launch_box(hipStream_t s, const LevelView<T>& L, const T* r, T* w, int colour, bool ib);
// ib_rows: evaluate the elastic rows first when the level has them (false
// only to time the box launch alone)
template <typename T> void launch_phase_fused(hipStream_t s, const LevelView<T>& L, const T* b, T* w, int colour,
                                              bool ib, bool ib_rows = true);
// A colour phase may run as one box launch that forms its own Stokes residuals
// (launch_phase_fused) when boxes of one colour are two boxes apart.
inline bool phase_fusable(int ncol, int n) { return ncol == 4 && (n == 2 || n == 4); }
// yf (nullable): elastic term of the fine residual (rf - yf is restricted)
template <typename T> void launch_restrict(hipStream_t s, int Nf, const T* rf, T* rc, T* wc_zero,
                                           const T* yf = nullptr, int walls = 0);
template <typename T> void launch_prolong_add(hipStream_t s, int Nf, const T* ec, T* wf, int walls = 0);
int prepare_tail(size_t lds);
template <typename T> int launch_tail(hipStream_t s, const LevelView<T>* views, int ls, int L, int nu1, int nu2,
                                      bool ib, int nr, const T* b_in, T* w_out, const double* cainv);
// walls: the cavity's wall faces and lid term (mu the viscosity); 0: periodic
void launch_rhs(hipStream_t s, const PointView& P, double c, double inv_h2, const double* u, const double* v,
                const double* gu, const double* gv, const double* G, double* b, int walls = 0, double mu = 0.0);
void launch_interp(hipStream_t s, const PointView& P, const double* u, const double* v, double* U,
                   double* X, double dt);

// dense.hip: bordered coarsest system
void launch_coarse_assemble(hipStream_t s, const LevelView<double>& L, double* aug, int nr);
int coarse_factor(hipStream_t s, double* aug, int nr, double* m, int* piv, double* dpiv, int* rowpos,
                  int* used, double* Y, double* ainv);
template <typename T> void launch_coarse_apply(hipStream_t s, const double* ainv, int nr, const T* b, T* w);

// krylov.hip
void launch_multidot(hipStream_t s, const double* V, size_t ldv, int nvec, const double* w, size_t n,
                     double* partial, int nblocks);
void launch_reduce(hipStream_t s, const double* partial, int nblocks, int nvec, double* out, int accumulate);
void launch_update(hipStream_t s, const double* V, size_t ldv, int nvec, const double* coef, double* w,
                   size_t n, double sign);
void launch_scale(hipStream_t s, const double* w, double* out, size_t n, const double* norm2);
void launch_givens(hipStream_t s, double* H, int ldh, double* g, double* cs, double* sn, int j, double* flags,
                   double target);
void launch_backsolve(hipStream_t s, const double* H, int ldh, const double* g, int k, double* y);
void launch_mean_shift(hipStream_t s, double* p, size_t n, const double* sum);
void launch_sum(hipStream_t s, const double* x, size_t n, double* partial, int nblocks);
void launch_reduce2(hipStream_t s, const double* partial, int nblocks, double* out, double* copy);
void launch_update_acc(hipStream_t s, const double* V, size_t ldv, int nvec, const double* coef, double* w, size_t n,
                       double* acc);
void launch_scale_givens(hipStream_t s, double* w, size_t n, const double* nrm2, double* H, int ldh, double* g,
                         double* cs, double* sn, int j, double* flags, double target);
// delayed CGS2 (krylov.hip): the products of V[0 .. nvec-1] with r1 and r2 in
// one pass (2 nvec dots, r2's after r1's); the coefficients and column
// completion; the update pass (partial = one |w'|^2 share per workgroup of
// nblk(n)); the scaling of u_{j+1} with the stopping test on a rotated copy
void launch_multidot2(hipStream_t s, const double* V, size_t ldv, int nvec, const double* r1, const double* r2,
                      size_t n, double* partial, int nblocks);
void launch_dcgs2_coef(hipStream_t s, const double* a, const double* c, int jf, double* H, int ldh, double* cs,
                       double* sn, double* g, double* coef);
void launch_dcgs2_update(hipStream_t s, double* V, size_t ldv, int j, const double* t, const double* sc,
                         const double* coef, size_t n, double* partial);
void launch_scale_tentative(hipStream_t s, double* w, size_t n, const double* nrm2, double* H, int ldh,
                            const double* g, const double* cs, const double* sn, int j, double* flags,
                            double target);

}  // namespace ibmg
