// Internal definitions shared by the gfx950 kernels and the host code of the
// implicit immersed-boundary multigrid library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define IBMG_MAX_LEVELS 12
#define IBMG_MAX_NDOF 56      // 2 n (n + 1) + n^2 for box edge n <= 4
#define IBMG_PATCH 16         // 4 x 4 per-point patch on every level

#define IBMG_WR 5                          // window reach on the finest level
#define IBMG_WW (2 * IBMG_WR + 1)          // window width
#define IBMG_WS (IBMG_WW * IBMG_WW)        // window entries per row

// Per-level view handed to kernels by value.  T is the precision of the
// V-cycle fields (double or float); box inverses of boxes that touch the
// structure and the coarsest inverse are always FP64.
//
// The elasticity block M_l of level l is held as one coefficient window per
// "active" velocity face (a face some row of M_l may reach): row f of M_l
// couples f to the faces f + (dx, dy), |dx|, |dy| <= reach, with coefficient
// win[(dy + WR) * WW + dx + WR].  The elimination factor -dt K (Sec. 2.3.2)
// is folded in.
template <typename T>
struct LevelView {
  int N;          // cells per side on this level (power of two)
  int nb;         // boxes per side
  int n;          // box edge in cells
  int ndof;       // unknowns per box
  int ncol;       // colour classes of a sweep (2 or 4)
  T c;            // rho / dt
  T muh2;         // mu / h_l^2
  T invh;         // 1 / h_l
  T omega;        // weight of a box correction (1: the undamped boxes of the paper)
  int walls;      // 0: periodic; 1: walls on all four sides (the cavity of Sec. 4).  With walls the
                  // faces u[j][0] (x = 0, standing for x = 1 too) and v[0][i] (y = 0 and y = 1) are
                  // identity rows that no other row reads; a face next to a wall parallel to it sees
                  // the ghost -u across it (the wall value is the average of face and ghost)
  int reach;      // window reach on this level
  int maxact;     // row capacity of the window store per component
  int rowhint;    // launch size of the elastic-row passes: expected active rows per component (<= maxact;
                  // the passes stride over the device-side count, so any size is correct)
  const int* act; // [2][N^2] active-row index of each face, or -1
  const T* win;   // [2][maxact][WS] windows
  const int* rows;// [2][maxact] face of each active row
  const int* nact;// [2] active rows per component
  T* yib;         // [2][N^2] (M_l w) on the active rows, zero elsewhere; formed before each colour phase
  const int* crow;   // levels whose four-colour phases run as one launch: [4][2][maxact] the active rows
                     // (indices into rows) lying in boxes of each colour, or null
  const int* ncrow;  // [4][2] their counts
  const int* ib_index;  // [nb^2] index of the box among boxes with elastic rows, or -1
  const T* ainv_plain;  // [ndof * ndof] inverse of the plain box block, column-major
  const double* ainv_ib;// [n_ib][ndof * ndof] inverses of boxes with elastic rows, column-major
};

// Finest-level Lagrangian data: delta-weight patches and point-to-box bins.
struct PointView {
  int M, N, n, nb;
  const int* prev;       // [M] fibre neighbours
  const int* next;       // [M]
  const int* org;        // [2][M][2] origin (i0, j0) of the 4 x 4 patch per component
  const double* wts;     // [2][M][16] phi(x) phi(y) per patch entry, x fastest
  const int* box_start;  // [nb^2 + 1] CSR of points whose patch meets each box
  const int* box_list;   // point ids, ascending within a box
};

__host__ __device__ inline int wrapi(int i, int N) { return i & (N - 1); }

// Peskin's 4-point kernel (kind 0) and the cosine 4-point kernel (kind 1),
// r in grid units (Sec. 2.2 regularised delta).
__device__ inline double phi_kernel(double r, int kind) {
  r = fabs(r);
  if (kind == 0) {
    if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(fmax(1.0 + 4.0 * r - 4.0 * r * r, 0.0))) * 0.125;
    if (r < 2.0) return (5.0 - 2.0 * r - sqrt(fmax(-7.0 + 12.0 * r - 4.0 * r * r, 0.0))) * 0.125;
    return 0.0;
  }
  if (r < 2.0) return 0.25 * (1.0 + cos(1.5707963267948966 * r));
  return 0.0;
}

// Workgroups (256 lanes, 16 rows each) striding over the active elastic rows
// of one component, and of both in the fused residual kernel.
__host__ __device__ inline int ib_blocks(int maxact) {
  const int b = (maxact * 16 + 255) / 256;
  return b < 512 ? b : 512;
}

// q-th box of a colour class.  ncol = 2: checkerboard, colour = (bx + by) & 1,
// nb * nb / 2 boxes per colour; ncol = 4: colour = (bx & 1) + 2 (by & 1),
// (nb / 2)^2 boxes per colour.  Row-major within a colour.
__host__ __device__ inline int colour_count(int ncol, int nb) { return ncol == 2 ? nb * (nb / 2) : (nb / 2) * (nb / 2); }
__host__ __device__ inline void colour_box(int q, int colour, int ncol, int nb, int& bx, int& by) {
  const int half = nb / 2;
  if (ncol == 2) {
    by = q / half;
    bx = 2 * (q - by * half) + ((by + colour) & 1);
  } else {
    bx = 2 * (q % half) + (colour & 1);
    by = 2 * (q / half) + (colour >> 1);
  }
}

// Local unknown r of box (bx, by) -> (component, i, j) on an N grid.
// Order: u faces (n+1 per row, n rows), v faces (n per row, n+1 rows),
// pressures (n x n), x fastest.
__device__ inline void box_dof(int r, int bx, int by, int n, int N, int& comp, int& i, int& j) {
  const int nu = n * (n + 1);
  if (r < nu) {
    comp = 0; i = bx * n + r % (n + 1); j = by * n + r / (n + 1);
  } else if (r < 2 * nu) {
    const int q = r - nu;
    comp = 1; i = bx * n + q % n; j = by * n + q / n;
  } else {
    const int q = r - 2 * nu;
    comp = 2; i = bx * n + q % n; j = by * n + q / n;
  }
  i = wrapi(i, N);
  j = wrapi(j, N);
}

// Inverse of box_dof: local index of (comp, i, j) in box (bx, by) or -1.
__device__ inline int box_local(int comp, int i, int j, int bx, int by, int n, int N) {
  const int li = wrapi(i - bx * n, N), lj = wrapi(j - by * n, N);
  const int nu = n * (n + 1);
  if (comp == 0) return (li <= n && lj < n) ? lj * (n + 1) + li : -1;
  if (comp == 1) return (li < n && lj <= n) ? nu + lj * n + li : -1;
  return (li < n && lj < n) ? 2 * nu + lj * n + li : -1;
}

// (A_l w) at one unknown without the elasticity term: unsteady Stokes on the
// MAC grid (Sec. 2.2) -- momentum c u - mu Lap u + G p, continuity -D u.
// With walls (L.walls): the walled rows described at LevelView::walls.
template <typename T>
__device__ inline T stokes_row_walls(const LevelView<T>& L, const T* __restrict__ w, int comp, int i, int j) {
  const int N = L.N, NN = N * N;
  const T* u = w;
  const T* v = w + NN;
  const T* p = w + 2 * NN;
  if (comp == 2) {
    const T ue = i + 1 < N ? u[j * N + i + 1] : T(0), uw = i > 0 ? u[j * N + i] : T(0);
    const T vn = j + 1 < N ? v[(j + 1) * N + i] : T(0), vs = j > 0 ? v[j * N + i] : T(0);
    return -((ue - uw) + (vn - vs)) * L.invh;
  }
  // a: index along the face normal (i for u), t: along the tangent
  const T* f = comp == 0 ? u : v;
  const int a = comp == 0 ? i : j, t = comp == 0 ? j : i;
  const int sa = comp == 0 ? 1 : N, st = comp == 0 ? N : 1;   // strides along a and t
  const int k = j * N + i;
  if (a == 0) return f[k];                                    // wall face: identity row
  const T c0 = f[k];
  T nb = T(0), ghosts = T(0);
  if (a + 1 < N) nb += f[k + sa];
  if (a - 1 > 0) nb += f[k - sa];
  if (t + 1 < N) nb += f[k + st]; else ghosts += T(1);
  if (t > 0) nb += f[k - st]; else ghosts += T(1);
  const T grad = (p[k] - p[k - sa]) * L.invh;
  return (L.c + (T(4) + ghosts) * L.muh2) * c0 - L.muh2 * nb + grad;
}

template <typename T>
__device__ inline T stokes_row(const LevelView<T>& L, const T* __restrict__ w, int comp, int i, int j) {
  if (L.walls) return stokes_row_walls(L, w, comp, i, j);
  const int N = L.N, NN = N * N;
  const T* u = w;
  const T* v = w + NN;
  const T* p = w + 2 * NN;
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  if (comp == 0) {
    const T c0 = u[j * N + i];
    const T nb = u[j * N + ip] + u[j * N + im] + u[jp * N + i] + u[jm * N + i];
    return (L.c + T(4) * L.muh2) * c0 - L.muh2 * nb + (p[j * N + i] - p[j * N + im]) * L.invh;
  } else if (comp == 1) {
    const T c0 = v[j * N + i];
    const T nb = v[j * N + ip] + v[j * N + im] + v[jp * N + i] + v[jm * N + i];
    return (L.c + T(4) * L.muh2) * c0 - L.muh2 * nb + (p[j * N + i] - p[jm * N + i]) * L.invh;
  }
  return -((u[j * N + ip] - u[j * N + i]) + (v[jp * N + i] - v[j * N + i])) * L.invh;
}

// Elasticity term (M_l w) at a velocity face from its coefficient window.
template <typename T>
__device__ inline T win_face(const LevelView<T>& L, const T* __restrict__ w, int comp, int i, int j) {
  const int N = L.N, msk = N - 1;
  const int a = L.act[comp * N * N + j * N + i];
  if (a < 0) return T(0);
  const T* c = L.win + ((size_t)comp * L.maxact + a) * IBMG_WS;
  const T* f = w + (size_t)comp * N * N;
  const int r = L.reach;
  T acc = T(0);
  for (int dy = -r; dy <= r; ++dy) {
    const T* row = f + (size_t)((j + dy) & msk) * N;
    const T* cw = c + (dy + IBMG_WR) * IBMG_WW + IBMG_WR;
    for (int dx = -r; dx <= r; ++dx) acc += cw[dx] * row[(i + dx) & msk];
  }
  return acc;
}

// Host-side helpers -----------------------------------------------------------
#define IBMG_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return IBMG_EHIP;              \
  } while (0)
