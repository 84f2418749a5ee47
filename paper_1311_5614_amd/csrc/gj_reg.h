// Gauss-Jordan inversion with partial pivoting of a dense block of up to
// 224 x 224 held in the registers of one 512-lane workgroup: lane
// (ty, tx) = (tid / 32, tid % 32) owns the 14 x 7 tile of rows 14 ty .. 14 ty + 13
// and columns 7 tx .. 7 tx + 6 (196 registers of the 256 a lane has at two
// waves per SIMD).  Used where the block is too large for the
// LDS form of gj.h: the 208-unknown blocks of 8 x 8 boxes (Sec. 6) and the
// bordered coarsest system of an 8 x 8 grid (193 unknowns, Algorithm 1).
//
// Step k pivots column k on the unused row p with the largest magnitude
// (lowest row on ties; a NaN counts as largest, so p is always an unused row
// and the pivot rows form a permutation) and applies the exchange ("sweep")
// operation in place,
// without moving rows:
//   a[p][k] <- 1 / d,  a[p][j] <- a[p][j] / d,  a[i][k] <- -a[i][k] / d,
//   a[i][j] <- a[i][j] - a[i][k] a[p][j] / d   (d = a[p][k]).
// After nd steps the tile holds the inverse with rows and columns permuted:
// with piv[k] the pivot row of column k and pinv its inverse permutation,
// A^{-1}[pinv[i]][piv[m]] = a[i][m].  Column k and pivot row p are exchanged
// through LDS (double-buffered by step parity, so a step needs two barriers).
#pragma once
#include <hip/hip_runtime.h>

constexpr int kGjTR = 14, kGjTC = 7, kGjGY = 16, kGjGX = 32, kGjMax = kGjTR * kGjGY;   // 224 = kGjTC * kGjGX
constexpr int kGjLanes = kGjGY * kGjGX;

struct GjScratch {
  double col[2][kGjMax];
  double row[2][kGjMax];
  double cv[2][kGjGY];
  int ci[2][kGjGY];
  int used[kGjMax];
  int piv[kGjMax];
  int pinv[kGjMax];
};

// load(i, j) -> A[i][j] for i, j < nd; store(r, c, v) receives A^{-1}[r][c].
// Every lane of the kGjLanes-lane workgroup must call this.
template <typename Load, typename Store>
__device__ inline void gauss_jordan_regs(int nd, GjScratch& S, Load load, Store store) {
  const int tid = threadIdx.x, tx = tid & (kGjGX - 1), ty = tid >> 5;
  const int r0 = ty * kGjTR, c0 = tx * kGjTC;
  double a[kGjTR][kGjTC];
#pragma unroll
  for (int r = 0; r < kGjTR; ++r)
#pragma unroll
    for (int c = 0; c < kGjTC; ++c)
      a[r][c] = (r0 + r < nd && c0 + c < nd) ? load(r0 + r, c0 + c) : 0.0;
  for (int i = tid; i < kGjMax; i += blockDim.x) S.used[i] = i >= nd;
  __syncthreads();
  for (int k = 0; k < nd; ++k) {
    const int b = k & 1, kt = k / kGjTC, kc = k - kt * kGjTC;
    // the lanes owning column k publish it and their best unused row
    if (tx == kt) {
      double bv = -1.0;
      int bi = kGjMax;
#pragma unroll
      for (int r = 0; r < kGjTR; ++r) {
        double v = a[r][0];
#pragma unroll
        for (int c = 1; c < kGjTC; ++c) v = kc == c ? a[r][c] : v;
        const int i = r0 + r;
        S.col[b][i] = v;
        const double m = fabs(v) == fabs(v) ? fabs(v) : INFINITY;   // a NaN row is taken, not skipped
        if (!S.used[i] && m > bv) { bv = m; bi = i; }
      }
      S.cv[b][ty] = bv;
      S.ci[b][ty] = bi;
    }
    __syncthreads();
    // every lane reduces the candidates in the same order (ties: lowest row)
    double bv = S.cv[b][0];
    int p = S.ci[b][0];
    for (int q = 1; q < kGjGY; ++q) {
      const double v = S.cv[b][q];
      if (v > bv) { bv = v; p = S.ci[b][q]; }
    }
    const int pt = p / kGjTR, pr = p - pt * kGjTR;
    if (ty == pt) {
#pragma unroll
      for (int r = 0; r < kGjTR; ++r)
        if (r == pr) {
#pragma unroll
          for (int c = 0; c < kGjTC; ++c) S.row[b][c0 + c] = a[r][c];
        }
    }
    if (tid == 0) {
      S.used[p] = 1;
      S.piv[k] = p;
    }
    __syncthreads();
    const double inv = 1.0 / S.col[b][p];
    double pj[kGjTC];
#pragma unroll
    for (int c = 0; c < kGjTC; ++c) pj[c] = S.row[b][c0 + c] * inv;
#pragma unroll
    for (int r = 0; r < kGjTR; ++r) {
      const int i = r0 + r;
      const double f = S.col[b][i];
#pragma unroll
      for (int c = 0; c < kGjTC; ++c) {
        const int j = c0 + c;
        if (i == p) a[r][c] = j == k ? inv : pj[c];
        else a[r][c] = j == k ? -f * inv : a[r][c] - f * pj[c];
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < nd; k += blockDim.x) S.pinv[S.piv[k]] = k;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kGjTR; ++r)
#pragma unroll
    for (int c = 0; c < kGjTC; ++c)
      if (r0 + r < nd && c0 + c < nd) store(S.pinv[r0 + r], S.piv[c0 + c], a[r][c]);
}
