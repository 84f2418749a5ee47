// Internal definitions shared by the gfx950 kernels and the host code of the
// implicit immersed-boundary multigrid library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define IBMG_MAX_LEVELS 12
#define IBMG_MAX_NDOF 56      // 2 n (n + 1) + n^2 for box edge n <= 4
#define IBMG_PATCH 16         // 4 x 4 per-point patch on every level

// Per-level view handed to kernels by value.  T is the precision of the
// V-cycle fields (double or float); box inverses of boxes that touch the
// structure and the coarsest inverse are always FP64.
template <typename T>
struct LevelView {
  int N;          // cells per side on this level (power of two)
  int nb;         // boxes per side
  int n;          // box edge in cells
  int ndof;       // unknowns per box
  T c;            // rho / dt
  T muh2;         // mu / h_l^2
  T invh;         // 1 / h_l
  T kappa;        // -dt K / h_0^2  (elasticity factor, Sec. 2.3.2 elimination)
  int M;          // Lagrangian points
  const int* prev;      // [M] fibre neighbours
  const int* next;      // [M]
  const int* orgB;      // [2][M][2] patch origins of the restricted spreading weights
  const T* wB;          // [2][M][16]
  const int* orgC;      // [2][M][2] patch origins of the prolonged interpolation weights
  const T* wC;          // [2][M][16]
  T* t;                 // [2][M] interpolated values C_l w
  const int* box_start; // [nb^2 + 1] CSR of points whose B patch meets each box
  const int* box_list;  // point ids, ascending within a box
  const int* ib_index;  // [nb^2] index of the box among boxes with points, or -1
  const T* ainv_plain;  // [ndof * ndof] inverse of the plain box block, column-major
  const double* ainv_ib;// [n_ib][ndof * ndof] inverses of boxes with points, column-major
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
template <typename T>
__device__ inline T stokes_row(const LevelView<T>& L, const T* __restrict__ w, int comp, int i, int j) {
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

// Elasticity term (M_l w) at a velocity face: kappa * sum over points k whose
// restricted spreading patch covers the face of B_l[k](face) * (L t)_k, with
// t = C_l w gathered beforehand.  Points come from the face's box list in
// ascending id order, so the sum is deterministic.
template <typename T>
__device__ inline T ib_face(const LevelView<T>& L, int comp, int i, int j) {
  const int box = (j / L.n) * L.nb + (i / L.n);
  const int s = L.box_start[box], e = L.box_start[box + 1];
  if (s == e) return T(0);
  const int msk = L.N - 1;
  const T* tt = L.t + comp * L.M;
  const int* org = L.orgB + comp * L.M * 2;
  const T* wb = L.wB + (size_t)comp * L.M * IBMG_PATCH;
  T acc = T(0);
  for (int q = s; q < e; ++q) {
    const int k = L.box_list[q];
    const int di = (i - org[2 * k]) & msk, dj = (j - org[2 * k + 1]) & msk;
    if (di < 4 && dj < 4) {
      const T sk = tt[L.prev[k]] - T(2) * tt[k] + tt[L.next[k]];
      acc += wb[k * IBMG_PATCH + dj * 4 + di] * sk;
    }
  }
  return L.kappa * acc;
}

// Host-side helpers -----------------------------------------------------------
#define IBMG_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return IBMG_EHIP;              \
  } while (0)
