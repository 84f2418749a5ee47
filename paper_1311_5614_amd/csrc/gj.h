// Gauss-Jordan inversion with partial pivoting of a small dense block held in
// LDS as the augmented [A | I] (row-major, nd rows, ld = 2 nd columns), one
// thread per column.  Per pivot step, wave 0 picks the pivot (largest
// magnitude in the column, ties to the lowest row) and snapshots the pivot
// column; then every thread swaps, scales and eliminates its own column only,
// so a step needs two barriers and no thread touches another's data.  On
// exit the right half holds A^{-1} (rows in natural order).  Used for the
// box blocks of the smoother (Sec. 5-6) and the small bordered coarsest
// system (Algorithm 1).
#pragma once
#include <hip/hip_runtime.h>

__device__ inline void gauss_jordan_cols(double* __restrict__ a, int nd, int ld, double* __restrict__ colk,
                                         int* __restrict__ piv, double* __restrict__ pval) {
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
      for (int i = tid; i < nd; i += 64) colk[i] = a[i * ld + k];
      if (tid == 0) {
        *piv = bi;
        *pval = a[bi * ld + k];
      }
    }
    __syncthreads();
    // columns left of k are already unit columns: row k holds 0 there.  Each
    // thread updates its own column; rows go eight at a time so that the LDS
    // accesses of a group are independent.
    const int p = *piv;
    const double inv = 1.0 / *pval, ck = colk[k];
    for (int c = k + tid; c < ld; c += blockDim.x) {
      const double ak = a[k * ld + c], ap = a[p * ld + c];
      const double nk = ap * inv;
      a[p * ld + c] = ak;
      a[k * ld + c] = nk;
      int i = 0;
      for (; i + 8 <= nd; i += 8) {
        double v[8], f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          v[u] = a[(i + u) * ld + c];
          f[u] = colk[i + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int ii = i + u;
          if (ii == k) continue;
          a[ii * ld + c] = v[u] - (ii == p ? ck : f[u]) * nk;
        }
      }
      for (; i < nd; ++i) {
        if (i == k) continue;
        const double f = i == p ? ck : colk[i];
        a[i * ld + c] -= f * nk;
      }
    }
    __syncthreads();
  }
}
