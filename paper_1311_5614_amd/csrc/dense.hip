// Exact coarsest-grid solve of Algorithm 1 (Sec. 3) on gfx950.
//
// The periodic coarsest system is singular in the pressure constant, so it
// is bordered: [[A_c, e_p], [e_p^T, 0]] (e_p = 1 on pressures), which fixes a
// zero-mean pressure.  The bordered matrix (size nr = 3 N_c^2 + 1) is
// assembled on the device (re-discretised Stokes plus the Galerkin elasticity
// block, Sec. 3.2) and inverted once per setup by blocked Gauss-Jordan with
// partial pivoting: a single-workgroup panel step picks PW pivots and the
// eliminated pivot-row values, then a grid-wide rank-PW update applies them
// to every other column.  Each V-cycle applies the inverse as a matrix-vector
// product.
#include "common.h"
#include "gj.h"
#include "gj_reg.h"
#include "kernels.h"

#define PW 16   // panel width

// Row r of the augmented [A_bordered | I], ld = 2 nr, one thread per row.
__global__ void __launch_bounds__(256)
k_coarse_assemble(LevelView<double> L, double* __restrict__ aug, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const int N = L.N, NN = N * N, msk = N - 1;
  const size_t ld = 2 * (size_t)nr;
  double* row = aug + (size_t)r * ld;
  for (size_t c = 0; c < ld; ++c) row[c] = 0.0;
  row[nr + r] = 1.0;
  if (r == nr - 1) {            // border row: sum of pressures
    for (int c = 2 * NN; c < 3 * NN; ++c) row[c] = 1.0;
    return;
  }
  const int comp = r / NN, rem = r - comp * NN;
  const int j = rem / N, i = rem - j * N;
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  const int base = comp * NN;
  if (L.walls) {   // the walled rows of stokes_row_walls
    if (comp < 2) {
      const int an = comp == 0 ? i : j, at = comp == 0 ? j : i;
      const int sa = comp == 0 ? 1 : N, st = comp == 0 ? N : 1;
      const int k = j * N + i;
      if (an == 0) {
        row[r] += 1.0;
        return;
      }
      const int ghosts = (at + 1 < N ? 0 : 1) + (at > 0 ? 0 : 1);
      row[r] += L.c + (4.0 + ghosts) * L.muh2;
      if (an + 1 < N) row[base + k + sa] -= L.muh2;
      if (an - 1 > 0) row[base + k - sa] -= L.muh2;
      if (at + 1 < N) row[base + k + st] -= L.muh2;
      if (at > 0) row[base + k - st] -= L.muh2;
      row[2 * NN + k] += L.invh;
      row[2 * NN + k - sa] -= L.invh;
      const int ar = L.act ? L.act[comp * NN + k] : -1;
      if (ar >= 0) {
        const double* cw = L.win + ((size_t)comp * L.maxact + ar) * IBMG_WS;
        for (int dy = -L.reach; dy <= L.reach; ++dy)
          for (int dx = -L.reach; dx <= L.reach; ++dx)
            row[base + ((j + dy) & msk) * N + ((i + dx) & msk)] += cw[(dy + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
      }
    } else {
      if (i + 1 < N) row[j * N + i + 1] -= L.invh;
      if (i > 0) row[j * N + i] += L.invh;
      if (j + 1 < N) row[NN + (j + 1) * N + i] -= L.invh;
      if (j > 0) row[NN + j * N + i] += L.invh;
      row[nr - 1] = 1.0;          // border column
    }
    return;
  }
  if (comp < 2) {
    row[r] += L.c + 4.0 * L.muh2;
    row[base + j * N + ip] -= L.muh2;
    row[base + j * N + im] -= L.muh2;
    row[base + jp * N + i] -= L.muh2;
    row[base + jm * N + i] -= L.muh2;
    row[2 * NN + j * N + i] += L.invh;
    if (comp == 0) row[2 * NN + j * N + im] -= L.invh;
    else row[2 * NN + jm * N + i] -= L.invh;
    const int ar = L.act ? L.act[comp * NN + j * N + i] : -1;
    if (ar >= 0) {
      const double* cw = L.win + ((size_t)comp * L.maxact + ar) * IBMG_WS;
      for (int dy = -L.reach; dy <= L.reach; ++dy)
        for (int dx = -L.reach; dx <= L.reach; ++dx)
          row[base + ((j + dy) & msk) * N + ((i + dx) & msk)] += cw[(dy + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
    }
  } else {
    row[j * N + ip] -= L.invh;
    row[j * N + i] += L.invh;
    row[NN + jp * N + i] -= L.invh;
    row[NN + j * N + i] += L.invh;
    row[nr - 1] = 1.0;          // border column
  }
}

// Panel step for columns k0..k0+PW-1.  Pivots are taken among rows not yet
// used (largest magnitude, lowest index on ties).  Records per panel column s:
// pivot row piv[k0+s], multipliers m[i][s] (row i's panel entry just before
// step s) and rowpos[i] = s for pivot rows (else -1).  Then forms
// Y[s][c] = eliminated pivot-row values for every column c >= k0+PW.  The
// panel and the used-row flags live in LDS for the whole step.
__global__ void __launch_bounds__(1024)
k_coarse_panel(const double* __restrict__ aug, int nr, int k0, double* __restrict__ m, int* __restrict__ piv,
               int* __restrict__ rowpos, int* __restrict__ used, double* __restrict__ Y) {
  extern __shared__ double P[];   // nr x PW panel, then nr ints of "used" flags
  int* usedl = (int*)(P + (size_t)nr * PW);
  __shared__ double wv[16];
  __shared__ int wi[16];
  __shared__ int pivs[PW];
  __shared__ double ds[PW];
  const int tid = threadIdx.x;
  const size_t ld = 2 * (size_t)nr;
  const int pw = min(PW, nr - k0);
  for (int idx = tid; idx < nr * PW; idx += blockDim.x) {
    const int i = idx / PW, s = idx - i * PW;
    P[idx] = s < pw ? aug[(size_t)i * ld + k0 + s] : 0.0;
  }
  for (int i = tid; i < nr; i += blockDim.x) usedl[i] = used[i];
  __syncthreads();
  for (int s = 0; s < pw; ++s) {
    double bv = -1.0;
    int bi = nr;
    for (int i = tid; i < nr; i += blockDim.x) {
      if (usedl[i]) continue;
      const double v = fabs(P[i * PW + s]);
      if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if ((tid & 63) == 0) { wv[tid >> 6] = bv; wi[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b0 = wv[0];
      int i0 = wi[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (wv[w] > b0 || (wv[w] == b0 && wi[w] < i0)) { b0 = wv[w]; i0 = wi[w]; }
      usedl[i0] = 1;
      pivs[s] = i0;
      ds[s] = P[i0 * PW + s];
    }
    __syncthreads();
    const int p = pivs[s];
    const double d = ds[s];
    // eliminate the panel columns t > s (multiplier = current entry in column s)
    for (int idx = tid; idx < nr * PW; idx += blockDim.x) {
      const int i = idx / PW, t = idx - i * PW;
      if (t <= s || i == p) continue;
      P[idx] -= P[i * PW + s] * (P[p * PW + t] / d);
    }
    __syncthreads();
    for (int t = s + 1 + tid; t < PW; t += blockDim.x) P[p * PW + t] /= d;
    __syncthreads();
  }
  // Column t < s of the panel still holds row i's multiplier for step t.
  for (int idx = tid; idx < nr * PW; idx += blockDim.x) {
    const int i = idx / PW, s = idx - i * PW;
    m[idx] = P[idx];
    (void)s;
  }
  for (int i = tid; i < nr; i += blockDim.x) {
    used[i] = usedl[i];
    int rp = -1;
    for (int s = 0; s < pw; ++s)
      if (pivs[s] == i) rp = s;
    rowpos[i] = rp;
  }
  if (tid < pw) piv[k0 + tid] = pivs[tid];
  // Y[s][c] for columns c >= k0 + pw: y_s = (a[p_s][c] - sum_{t<s} m[p_s][t] y_t) / d_s
  for (size_t c = k0 + pw + tid; c < ld; c += blockDim.x) {
    double y[PW];
    for (int s = 0; s < pw; ++s) {
      const int p = pivs[s];
      double v = aug[(size_t)p * ld + c];
      for (int t = 0; t < s; ++t) v -= P[p * PW + t] * y[t];
      y[s] = v / ds[s];
      Y[(size_t)s * ld + c] = y[s];
    }
  }
}

// Applies the panel's PW Gauss-Jordan steps to column c:
// a[i][c] -= sum_s m[i][s] Y[s][c] for non-pivot rows,
// a[p_s][c] = Y[s][c] - sum_{t>s} m[p_s][t] Y[t][c] for the pivot rows.
__global__ void __launch_bounds__(256)
k_coarse_update(double* __restrict__ aug, int nr, int k0, int pw, const double* __restrict__ m,
                const int* __restrict__ rowpos, const double* __restrict__ Y) {
  const size_t ld = 2 * (size_t)nr;
  const size_t c = (size_t)k0 + pw + (size_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (c >= ld) return;
  const int r0 = blockIdx.y * 4 + (threadIdx.x >> 6);
  double y[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) y[s] = s < pw ? Y[(size_t)s * ld + c] : 0.0;
  for (int i = r0; i < nr; i += gridDim.y * 4) {
    // pivot row p_s: y_s, then eliminated by the later pivots t > s of the
    // panel; any other row: eliminated by every pivot of the panel
    const int rp = rowpos[i];
    double* a = aug + (size_t)i * ld + c;
    const double* mi = m + (size_t)i * PW;
    double v = rp >= 0 ? 0.0 : *a;
#pragma unroll
    for (int s = 0; s < PW; ++s) {
      const double coef = (s < rp || s >= pw) ? 0.0 : (s == rp ? -1.0 : mi[s]);
      v -= coef * y[s];
    }
    *a = v;
  }
}

// inverse row c = right half of row piv[c] (the left block ended as a row
// permutation of the identity).
__global__ void __launch_bounds__(256)
k_coarse_gather(const double* __restrict__ aug, int nr, const int* __restrict__ piv, double* __restrict__ ainv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nr * nr) return;
  const int r = (int)(idx / nr), c = (int)(idx - (size_t)r * nr);
  ainv[idx] = aug[(size_t)piv[r] * 2 * nr + nr + c];
}

// w = first nr-1 entries of A^{-1} [b; 0]; one wave per row, fixed lane order.
template <typename T>
__global__ void __launch_bounds__(256)
k_coarse_apply(const double* __restrict__ ainv, int nr, const T* __restrict__ b, T* __restrict__ w) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nr - 1) return;
  const double* a = ainv + (size_t)row * nr;
  double acc = 0.0;
  for (int c = lane; c < nr - 1; c += 64) acc += a[c] * (double)b[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if (lane == 0) w[row] = (T)acc;
}

// Small bordered systems (nr <= IBMG_MAX_NDOF, e.g. the 4 x 4 coarsest grid):
// the whole augmented matrix in LDS, inverted by one workgroup.
__global__ void __launch_bounds__(128)
k_coarse_small(const double* __restrict__ aug, int nr, double* __restrict__ ainv) {
  __shared__ double a[IBMG_MAX_NDOF * 2 * IBMG_MAX_NDOF];
  __shared__ double colk[IBMG_MAX_NDOF];
  __shared__ int piv;
  __shared__ double pval;
  const int ld = 2 * nr;
  for (int idx = threadIdx.x; idx < nr * ld; idx += blockDim.x) a[idx] = aug[idx];
  __syncthreads();
  gauss_jordan_cols(a, nr, ld, colk, &piv, &pval);
  for (int idx = threadIdx.x; idx < nr * nr; idx += blockDim.x) {
    const int r = idx / nr, c = idx - r * nr;
    ainv[idx] = a[r * ld + nr + c];
  }
}

// Bordered systems of IBMG_MAX_NDOF < nr <= 224 (the 8 x 8 coarsest grid):
// the left half of the augmented matrix inverted in the registers of one
// workgroup (gj_reg.h); inverse row-major.
__global__ void __launch_bounds__(kGjLanes)
k_coarse_regs(const double* __restrict__ aug, int nr, double* __restrict__ ainv) {
  __shared__ GjScratch S;
  const size_t ld = 2 * (size_t)nr;
  gauss_jordan_regs(
      nr, S, [&](int i, int j) { return aug[(size_t)i * ld + j]; },
      [&](int r, int c, double v) { ainv[(size_t)r * nr + c] = v; });
}

namespace ibmg {

void launch_coarse_assemble(hipStream_t s, const LevelView<double>& L, double* aug, int nr) {
  k_coarse_assemble<<<nblk(nr), 256, 0, s>>>(L, aug, nr);
}

int coarse_factor(hipStream_t s, double* aug, int nr, double* m, int* piv, double* dpiv, int* rowpos,
                  int* used, double* Y, double* ainv) {
  (void)dpiv;
  if (nr <= IBMG_MAX_NDOF) {
    k_coarse_small<<<1, 128, 0, s>>>(aug, nr, ainv);
    return 0;
  }
  if (nr <= kGjMax) {
    k_coarse_regs<<<1, kGjLanes, 0, s>>>(aug, nr, ainv);
    return 0;
  }
  const size_t lds = (size_t)nr * PW * sizeof(double) + (size_t)nr * sizeof(int);
  if (lds > 65536 && hipFuncSetAttribute((const void*)k_coarse_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds) != hipSuccess)
    return -1;
  k_fill_i32<<<nblk(nr), 256, 0, s>>>(used, nr, 0);
  const size_t ld = 2 * (size_t)nr;
  for (int k0 = 0; k0 < nr; k0 += PW) {
    const int pw = nr - k0 < PW ? nr - k0 : PW;
    k_coarse_panel<<<1, 1024, lds, s>>>(aug, nr, k0, m, piv, rowpos, used, Y);
    const size_t ncols = ld - (size_t)(k0 + pw);
    if (ncols > 0) {
      dim3 grid((unsigned)((ncols + 63) / 64), 16);
      k_coarse_update<<<grid, 256, 0, s>>>(aug, nr, k0, pw, m, rowpos, Y);
    }
  }
  k_coarse_gather<<<nblk((size_t)nr * nr), 256, 0, s>>>(aug, nr, piv, ainv);
  return 0;
}

template <typename T> void launch_coarse_apply(hipStream_t s, const double* ainv, int nr, const T* b, T* w) {
  k_coarse_apply<T><<<nblk(nr - 1, 4), 256, 0, s>>>(ainv, nr, b, w);
}
template void launch_coarse_apply<double>(hipStream_t, const double*, int, const double*, double*);
template void launch_coarse_apply<float>(hipStream_t, const double*, int, const float*, float*);

}  // namespace ibmg
