// Per-step operator setup on gfx950: fibre forces, delta weights, Galerkin-
// coarsened per-point patches, point-to-box binning and dense box factors.
//
// Paper references: fibre force and regularised delta (Sec. 2.2), lagged
// spreading/interpolation (Sec. 2.3.2), Galerkin coarsening of the
// elasticity operator with the Sec. 3.1 transfers (Sec. 3.2), box relaxation
// blocks (Sec. 5-6) and the observation that plain boxes share one factor
// while boxes near the structure need their own, re-formed every step (Sec. 8).
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------- a1: G = K L X
__global__ void __launch_bounds__(256)
k_fiber_force(int M, const int* __restrict__ prev, const int* __restrict__ next, double K,
              const double* __restrict__ X, double* __restrict__ G) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const int a = prev[k], b = next[k];
  G[2 * k] = K * (X[2 * a] - 2.0 * X[2 * k] + X[2 * b]);
  G[2 * k + 1] = K * (X[2 * a + 1] - 2.0 * X[2 * k + 1] + X[2 * b + 1]);
}

// ---------------------------------------------------------------- a3: finest patches
// Component 0 (u faces at (i, j + 1/2)) and 1 (v faces at (i + 1/2, j)), grid
// units.  The 4 x 4 patch starts at floor(s) - 1 in each direction, which
// contains the whole support |r| < 2 of either kernel.
__global__ void __launch_bounds__(256)
k_weights0(int M, int N, int kind, const double* __restrict__ X, int* __restrict__ org,
           double* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * M) return;
  const int comp = t / M, k = t % M;
  double sx = X[2 * k] * N, sy = X[2 * k + 1] * N;
  if (comp == 0) sy -= 0.5; else sx -= 0.5;
  const double fx = floor(sx), fy = floor(sy);
  const int i0 = (int)fx - 1, j0 = (int)fy - 1;
  double wx[4], wy[4];
  for (int a = 0; a < 4; ++a) {
    wx[a] = phi_kernel((double)(i0 + a) - sx, kind);
    wy[a] = phi_kernel((double)(j0 + a) - sy, kind);
  }
  double* o = w + (size_t)t * IBMG_PATCH;
  for (int b = 0; b < 4; ++b)
    for (int a = 0; a < 4; ++a) o[b * 4 + a] = wx[a] * wy[b];
  org[2 * t] = ((i0 % N) + N) % N;
  org[2 * t + 1] = ((j0 % N) + N) % N;
}

// ---------------------------------------------------------------- a5: Galerkin patches
// B_{l+1} = R_l B_l (restriction of the spreading patch) and
// C_{l+1} = C_l P_l (interpolation patch through bilinear prolongation),
// evaluated on unwrapped relative offsets, so every coarse entry is a plain
// sum of fine entries.  New origins: B: (floor(a/2), floor(b/2));
// C: normal direction floor(a/2), tangential floor((b-1)/2).
struct PatchLevels {
  int* orgB[IBMG_MAX_LEVELS];
  double* wB[IBMG_MAX_LEVELS];
  int* orgC[IBMG_MAX_LEVELS];
  double* wC[IBMG_MAX_LEVELS];
  int N[IBMG_MAX_LEVELS];
};

__device__ inline int floordiv2(int a) { return a >> 1; }   // arithmetic shift floors

__global__ void __launch_bounds__(256)
k_coarsen(int M, int levels, PatchLevels P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * M) return;
  const int comp = t / M;
  const double wr[3] = {1.0 / 8.0, 2.0 / 8.0, 1.0 / 8.0};
  for (int l = 0; l + 1 < levels; ++l) {
    const int Nc = P.N[l + 1];
    // ---- restriction of B
    {
      const int a = P.orgB[l][2 * t], b = P.orgB[l][2 * t + 1];
      const double* f = P.wB[l] + (size_t)t * IBMG_PATCH;
      const int A0 = floordiv2(a), B0 = floordiv2(b);
      double out[16];
      for (int q = 0; q < 16; ++q) out[q] = 0.0;
      for (int J = 0; J < 4; ++J)
        for (int I = 0; I < 4; ++I) {
          double s = 0.0;
          for (int d = -1; d <= 1; ++d)
            for (int e = 0; e <= 1; ++e) {
              int fx, fy;
              if (comp == 0) { fx = 2 * (A0 + I) + d - a; fy = 2 * (B0 + J) + e - b; }
              else           { fx = 2 * (A0 + I) + e - a; fy = 2 * (B0 + J) + d - b; }
              if (fx >= 0 && fx < 4 && fy >= 0 && fy < 4) s += wr[d + 1] * f[fy * 4 + fx];
            }
          out[J * 4 + I] = s;
        }
      double* o = P.wB[l + 1] + (size_t)t * IBMG_PATCH;
      for (int q = 0; q < 16; ++q) o[q] = out[q];
      P.orgB[l + 1][2 * t] = wrapi(A0, Nc);
      P.orgB[l + 1][2 * t + 1] = wrapi(B0, Nc);
    }
    // ---- prolongation of C
    {
      const int a = P.orgC[l][2 * t], b = P.orgC[l][2 * t + 1];
      const double* f = P.wC[l] + (size_t)t * IBMG_PATCH;
      // normal direction (x for u, y for v) and tangential direction origins
      const int an = comp == 0 ? a : b;   // fine origin along the normal
      const int at = comp == 0 ? b : a;   // fine origin along the tangent
      const int N0 = floordiv2(an), T0 = floordiv2(at - 1);
      double out[16];
      for (int q = 0; q < 16; ++q) out[q] = 0.0;
      for (int fy = 0; fy < 4; ++fy)
        for (int fx = 0; fx < 4; ++fx) {
          const double val = f[fy * 4 + fx];
          const int in = comp == 0 ? an + fx : an + fy;   // fine index along normal
          const int it = comp == 0 ? at + fy : at + fx;   // fine index along tangent
          int cn[2], ct[2];
          double wn[2], wt[2];
          int nn, nt;
          if ((in & 1) == 0) { cn[0] = in >> 1; wn[0] = 1.0; nn = 1; }
          else { cn[0] = (in - 1) >> 1; cn[1] = (in + 1) >> 1; wn[0] = wn[1] = 0.5; nn = 2; }
          const int Jt = it >> 1;
          if ((it & 1) == 0) { ct[0] = Jt; wt[0] = 0.75; ct[1] = Jt - 1; wt[1] = 0.25; }
          else { ct[0] = Jt; wt[0] = 0.75; ct[1] = Jt + 1; wt[1] = 0.25; }
          nt = 2;
          for (int x = 0; x < nn; ++x)
            for (int y = 0; y < nt; ++y) {
              const int rn = cn[x] - N0, rt = ct[y] - T0;
              const int cx = comp == 0 ? rn : rt, cy = comp == 0 ? rt : rn;
              out[cy * 4 + cx] += val * wn[x] * wt[y];
            }
        }
      double* o = P.wC[l + 1] + (size_t)t * IBMG_PATCH;
      for (int q = 0; q < 16; ++q) o[q] = out[q];
      const int ox = comp == 0 ? N0 : T0, oy = comp == 0 ? T0 : N0;
      P.orgC[l + 1][2 * t] = wrapi(ox, Nc);
      P.orgC[l + 1][2 * t + 1] = wrapi(oy, Nc);
    }
  }
}

// ---------------------------------------------------------------- a2: point-to-box binning
__device__ inline void add_unique(int* a, int& n, int v) {
  for (int q = 0; q < n; ++q)
    if (a[q] == v) return;
  a[n++] = v;
}

// Boxes whose unknowns of component comp meet the 4 x 4 patch at (oi, oj).
// A u face on a box's left edge also belongs to the box on its left (shared
// edge unknowns are updated by both boxes, Sec. 6); likewise v in y.
__device__ inline void patch_boxes(int comp, int oi, int oj, int n, int N, int nb, int* ids, int& cnt) {
  int bxs[8], bys[8], nbx = 0, nby = 0;
  for (int a = 0; a < 4; ++a) {
    const int x = wrapi(oi + a, N), y = wrapi(oj + a, N);
    add_unique(bxs, nbx, x / n);
    if (comp == 0 && x % n == 0) add_unique(bxs, nbx, (x / n - 1 + nb) % nb);
    add_unique(bys, nby, y / n);
    if (comp == 1 && y % n == 0) add_unique(bys, nby, (y / n - 1 + nb) % nb);
  }
  for (int p = 0; p < nby; ++p)
    for (int q = 0; q < nbx; ++q) add_unique(ids, cnt, bys[p] * nb + bxs[q]);
}

__device__ inline int point_boxes(int k, int M, const int* orgB, int n, int N, int nb, int* ids) {
  int cnt = 0;
  for (int comp = 0; comp < 2; ++comp)
    patch_boxes(comp, orgB[(comp * M + k) * 2], orgB[(comp * M + k) * 2 + 1], n, N, nb, ids, cnt);
  return cnt;
}

__global__ void __launch_bounds__(256)
k_box_count(int M, const int* __restrict__ orgB, int n, int N, int nb, int* __restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  int ids[64];
  const int c = point_boxes(k, M, orgB, n, N, nb, ids);
  for (int q = 0; q < c; ++q) atomicAdd(&cnt[ids[q]], 1);
}

__global__ void __launch_bounds__(256)
k_box_fill(int M, const int* __restrict__ orgB, int n, int N, int nb, const int* __restrict__ start,
           int* __restrict__ cursor, int* __restrict__ list, int max_list) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  int ids[64];
  const int c = point_boxes(k, M, orgB, n, N, nb, ids);
  for (int q = 0; q < c; ++q) {
    const int pos = atomicAdd(&cursor[ids[q]], 1);
    const int at = start[ids[q]] + pos;
    if (at < max_list) list[at] = k;
  }
}

// Ascending point ids within each box (fixed summation order downstream).
__global__ void __launch_bounds__(256)
k_box_sort(int nbox, const int* __restrict__ start, int* __restrict__ list) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  const int s = start[b], e = start[b + 1];
  for (int i = s + 1; i < e; ++i) {
    const int v = list[i];
    int j = i - 1;
    while (j >= s && list[j] > v) { list[j + 1] = list[j]; --j; }
    list[j + 1] = v;
  }
}

// Block-wide exclusive scan helper (1024 threads).
__device__ inline int block_excl_scan(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int a = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  total = sh[1023];
  const int incl = sh[tid];
  __syncthreads();
  return incl - v;
}

// start[] = exclusive scan of cnt[]; cursor[] = 0.
__global__ void __launch_bounds__(1024)
k_scan_counts(int nbox, const int* __restrict__ cnt, int* __restrict__ start, int* __restrict__ cursor) {
  __shared__ int sh[1024];
  int base = 0;
  for (int c0 = 0; c0 < nbox; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int v = i < nbox ? cnt[i] : 0;
    int total;
    const int ex = block_excl_scan(v, sh, total);
    if (i < nbox) { start[i] = base + ex; cursor[i] = 0; }
    base += total;
  }
  if (threadIdx.x == 0) start[nbox] = base;
}

// Number the boxes that hold points, colour by colour ((0,0),(1,0),(0,1),(1,1)),
// row-major within a colour (nb >= 2, even).  ib_boxes[idx] = box id;
// info[c] = count of colour c; info[4] = total.
__global__ void __launch_bounds__(1024)
k_ib_index(int nb, const int* __restrict__ cnt, int* __restrict__ ib_index, int* __restrict__ ib_boxes,
           int* __restrict__ info) {
  __shared__ int sh[1024];
  const int colx[4] = {0, 1, 0, 1}, coly[4] = {0, 0, 1, 1};
  const int half = nb / 2, per = half * half;
  int base = 0;
  for (int c = 0; c < 4; ++c) {
    int cbase = base;
    for (int c0 = 0; c0 < per; c0 += 1024) {
      const int q = c0 + threadIdx.x;
      int box = 0, flag = 0;
      if (q < per) {
        box = (2 * (q / half) + coly[c]) * nb + 2 * (q % half) + colx[c];
        flag = cnt[box] > 0 ? 1 : 0;
      }
      int total;
      const int ex = block_excl_scan(flag, sh, total);
      if (q < per) {
        ib_index[box] = flag ? cbase + ex : -1;
        if (flag) ib_boxes[cbase + ex] = box;
      }
      cbase += total;
    }
    if (threadIdx.x == 0) info[c] = cbase - base;
    base = cbase;
  }
  if (threadIdx.x == 0) info[4] = base;
}

// ---------------------------------------------------------------- a6: box blocks
// Assemble A_l[box, box] (Stokes stencil restricted to the box plus the
// elasticity block kappa * sum_k B_k L C_k' over the box's points) into an
// LDS buffer with leading dimension ld.
__device__ void assemble_box(const LevelView<double>& L, int bx, int by, bool with_ib, double* a, int ld) {
  const int n = L.n, N = L.N, nd = L.ndof, msk = N - 1;
  for (int r = threadIdx.x; r < nd; r += blockDim.x) {
    int comp, i, j;
    box_dof(r, bx, by, n, N, comp, i, j);
    double* row = a + (size_t)r * ld;
    const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
    int col;
    if (comp < 2) {
      row[r] += L.c + 4.0 * L.muh2;
      const int nbi[4] = {ip, im, i, i}, nbj[4] = {j, j, jp, jm};
      for (int q = 0; q < 4; ++q)
        if ((col = box_local(comp, nbi[q], nbj[q], bx, by, n, N)) >= 0) row[col] -= L.muh2;
      if (comp == 0) {
        if ((col = box_local(2, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if ((col = box_local(2, im, j, bx, by, n, N)) >= 0) row[col] -= L.invh;
      } else {
        if ((col = box_local(2, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if ((col = box_local(2, i, jm, bx, by, n, N)) >= 0) row[col] -= L.invh;
      }
      if (with_ib) {
        const int box = by * L.nb + bx;
        const int* orgB = L.orgB + comp * L.M * 2;
        const int* orgC = L.orgC + comp * L.M * 2;
        const double* wB = L.wB + (size_t)comp * L.M * IBMG_PATCH;
        const double* wC = L.wC + (size_t)comp * L.M * IBMG_PATCH;
        for (int q = L.box_start[box]; q < L.box_start[box + 1]; ++q) {
          const int k = L.box_list[q];
          const int di = (i - orgB[2 * k]) & msk, dj = (j - orgB[2 * k + 1]) & msk;
          if (di >= 4 || dj >= 4) continue;
          const double bk = L.kappa * wB[k * IBMG_PATCH + dj * 4 + di];
          const int nbk[3] = {L.prev[k], k, L.next[k]};
          const double lc[3] = {1.0, -2.0, 1.0};
          for (int s = 0; s < 3; ++s) {
            const int kk = nbk[s];
            const int oi = orgC[2 * kk], oj = orgC[2 * kk + 1];
            for (int e = 0; e < 16; ++e) {
              const int ci = wrapi(oi + (e & 3), N), cj = wrapi(oj + (e >> 2), N);
              if ((col = box_local(comp, ci, cj, bx, by, n, N)) >= 0)
                row[col] += bk * lc[s] * wC[kk * IBMG_PATCH + e];
            }
          }
        }
      }
    } else {
      if ((col = box_local(0, ip, j, bx, by, n, N)) >= 0) row[col] -= L.invh;
      if ((col = box_local(0, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
      if ((col = box_local(1, i, jp, bx, by, n, N)) >= 0) row[col] -= L.invh;
      if ((col = box_local(1, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
    }
  }
}

// Gauss-Jordan with partial pivoting on [A | I] in LDS (ties -> lowest row).
__device__ void gauss_jordan_lds(double* a, int nd, int ld, double* colk, int* piv) {
  const int tid = threadIdx.x;
  for (int k = 0; k < nd; ++k) {
    if (tid < 64) {
      double bv = -1.0;
      int bi = nd;
      for (int i = k + tid; i < nd; i += 64) {
        const double v = fabs(a[i * ld + k]);
        if (v > bv) { bv = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (tid == 0) *piv = bi;
    }
    __syncthreads();
    const int p = *piv;
    if (p != k)
      for (int c = tid; c < ld; c += blockDim.x) {
        const double t = a[k * ld + c];
        a[k * ld + c] = a[p * ld + c];
        a[p * ld + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / a[k * ld + k];
    __syncthreads();
    for (int c = tid; c < ld; c += blockDim.x) a[k * ld + c] *= inv;
    for (int i = tid; i < nd; i += blockDim.x) colk[i] = a[i * ld + k];
    __syncthreads();
    for (int idx = tid; idx < nd * ld; idx += blockDim.x) {
      const int i = idx / ld, c = idx - i * ld;
      if (i != k && c >= k) a[idx] -= colk[i] * a[k * ld + c];
    }
    __syncthreads();
  }
}

// Block 0: the plain box (Stokes only, shared by every box without points).
// Block 1 + q: box ib_boxes[q].  Inverses are written column-major.
__global__ void __launch_bounds__(256)
k_box_factor(LevelView<double> L, const int* __restrict__ ib_boxes, double* __restrict__ ainv_plain,
             float* __restrict__ ainv_plain_f, double* __restrict__ ainv_ib) {
  __shared__ double a[IBMG_MAX_NDOF * 2 * IBMG_MAX_NDOF];
  __shared__ double colk[IBMG_MAX_NDOF];
  __shared__ int piv;
  const int nd = L.ndof, ld = 2 * nd;
  const bool plain = blockIdx.x == 0;
  int bx = 0, by = 0;
  if (!plain) {
    const int box = ib_boxes[blockIdx.x - 1];
    bx = box % L.nb;
    by = box / L.nb;
  }
  for (int idx = threadIdx.x; idx < nd * ld; idx += blockDim.x) {
    const int i = idx / ld, c = idx - i * ld;
    a[idx] = (c == nd + i) ? 1.0 : 0.0;
  }
  __syncthreads();
  assemble_box(L, bx, by, !plain, a, ld);
  __syncthreads();
  gauss_jordan_lds(a, nd, ld, colk, &piv);
  double* out = plain ? ainv_plain : ainv_ib + (size_t)(blockIdx.x - 1) * nd * nd;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) {
    const int r = idx / nd, c = idx - r * nd;
    const double v = a[r * ld + nd + c];
    out[c * nd + r] = v;
    if (plain && ainv_plain_f) ainv_plain_f[c * nd + r] = (float)v;
  }
}

// Assembled (not inverted) block of one box, row-major, for inspection.
__global__ void __launch_bounds__(256)
k_box_matrix(LevelView<double> L, int bx, int by, double* __restrict__ out) {
  __shared__ double a[IBMG_MAX_NDOF * IBMG_MAX_NDOF];
  const int nd = L.ndof;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) a[idx] = 0.0;
  __syncthreads();
  const int box = by * L.nb + bx;
  const bool ib = L.M > 0 && L.box_start[box + 1] > L.box_start[box];
  assemble_box(L, bx, by, ib, a, nd);
  __syncthreads();
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) out[idx] = a[idx];
}

// ---------------------------------------------------------------- launchers
namespace ibmg {

void launch_fiber_force(hipStream_t s, int M, const int* prev, const int* next, double K,
                        const double* X, double* G) {
  if (M > 0) k_fiber_force<<<(M + 255) / 256, 256, 0, s>>>(M, prev, next, K, X, G);
}

void launch_weights0(hipStream_t s, int M, int N, int kind, const double* X, int* org, double* w) {
  if (M > 0) k_weights0<<<(2 * M + 255) / 256, 256, 0, s>>>(M, N, kind, X, org, w);
}

void launch_coarsen(hipStream_t s, int M, int levels, int* const* orgB, double* const* wB,
                    int* const* orgC, double* const* wC, const int* Ns) {
  if (M == 0 || levels < 2) return;
  PatchLevels P;
  for (int l = 0; l < levels; ++l) {
    P.orgB[l] = orgB[l]; P.wB[l] = wB[l]; P.orgC[l] = orgC[l]; P.wC[l] = wC[l]; P.N[l] = Ns[l];
  }
  k_coarsen<<<(2 * M + 255) / 256, 256, 0, s>>>(M, levels, P);
}

void launch_box_lists(hipStream_t s, int M, const int* orgB, int n, int N, int nb, int* cnt, int* start,
                      int* cursor, int* list, int max_list, int* ib_index, int* ib_boxes, int* info) {
  const int nbox = nb * nb;
  k_fill_i32<<<(nbox + 255) / 256, 256, 0, s>>>(cnt, nbox, 0);
  if (M > 0) k_box_count<<<(M + 255) / 256, 256, 0, s>>>(M, orgB, n, N, nb, cnt);
  k_scan_counts<<<1, 1024, 0, s>>>(nbox, cnt, start, cursor);
  if (M > 0) {
    k_box_fill<<<(M + 255) / 256, 256, 0, s>>>(M, orgB, n, N, nb, start, cursor, list, max_list);
    k_box_sort<<<(nbox + 255) / 256, 256, 0, s>>>(nbox, start, list);
  }
  if (ib_index) k_ib_index<<<1, 1024, 0, s>>>(nb, cnt, ib_index, ib_boxes, info);
}

void launch_box_factor(hipStream_t s, const LevelView<double>& L, const int* ib_boxes, int n_ib,
                       double* ainv_plain, float* ainv_plain_f, double* ainv_ib) {
  k_box_factor<<<1 + n_ib, 256, 0, s>>>(L, ib_boxes, ainv_plain, ainv_plain_f, ainv_ib);
}

void launch_box_matrix(hipStream_t s, const LevelView<double>& L, int bx, int by, double* out) {
  k_box_matrix<<<1, 256, 0, s>>>(L, bx, by, out);
}

}  // namespace ibmg
