// Gauss-Jordan inversion with partial pivoting of a dense block of up to
// 224 x 224 held in the registers of one 512-lane workgroup: lane
// tid = 16 tx + ty owns the 14 x 7 tile of rows 14 ty .. 14 ty + 13 and
// columns 7 tx .. 7 tx + 6 (196 registers of the 256 a lane has at two waves
// per SIMD); the 16 lanes owning a column of tiles are adjacent lanes of one
// wave, so the pivot search is a shuffle reduction inside that wave.  Used
// where the block is too large for the LDS form of gj.h: the 208-unknown
// blocks of 8 x 8 boxes (Sec. 6) and the bordered coarsest system of an
// 8 x 8 grid (193 unknowns, Algorithm 1).
//
// Step k pivots column k on the unused row p with the largest magnitude
// (lowest row on ties; a NaN counts as largest, so p is always an unused row
// and the pivot rows form a permutation) and applies the exchange ("sweep")
// operation in place, without moving rows:
//   a[p][k] <- 1 / d,  a[p][j] <- a[p][j] / d,  a[i][k] <- -a[i][k] / d,
//   a[i][j] <- a[i][j] - a[i][k] a[p][j] / d   (d = a[p][k]).
// After nd steps the tile holds the inverse with rows and columns permuted:
// with piv[k] the pivot row of column k and pinv its inverse permutation,
// A^{-1}[pinv[i]][piv[m]] = a[i][m].  Column k goes through LDS (double-
// buffered by step parity); the pivot row is shuffled inside each 16-lane
// group, so a step needs one barrier.
#pragma once
#include <hip/hip_runtime.h>

constexpr int kGjTR = 14, kGjTC = 7, kGjGY = 16, kGjGX = 32;
constexpr int kGjMax = kGjTR * kGjGY;   // 224 rows = kGjTC * kGjGX columns
constexpr int kGjLanes = kGjGY * kGjGX;

struct GjScratch {
  double col[2][kGjMax];
  int p[2];
  int piv[kGjMax];
  int pinv[kGjMax];
};

// load(i, j) -> A[i][j] for i, j < nd; store(r, c, v) receives A^{-1}[r][c].
// Every lane of the kGjLanes-lane workgroup must call this.  The pivot row is
// made wave-uniform (readfirstlane) so that its tile row is picked by scalar
// branches; the tile column of k is picked by selects in the one wave that
// owns it.
template <typename Load, typename Store>
__device__ inline void gauss_jordan_regs(int nd, GjScratch& S, Load load, Store store) {
  const int tid = threadIdx.x, ty = tid & (kGjGY - 1), tx = tid >> 4;
  const int r0 = ty * kGjTR, c0 = tx * kGjTC;
  double a[kGjTR][kGjTC];
#pragma unroll
  for (int r = 0; r < kGjTR; ++r)
#pragma unroll
    for (int c = 0; c < kGjTC; ++c)
      a[r][c] = (r0 + r < nd && c0 + c < nd) ? load(r0 + r, c0 + c) : 0.0;
  unsigned used = 0;   // bit r: row r0 + r is a pivot row already (or past nd)
#pragma unroll
  for (int r = 0; r < kGjTR; ++r)
    if (r0 + r >= nd) used |= 1u << r;
  for (int k = 0; k < nd; ++k) {
    const int b = k & 1, kt = k / kGjTC, kc = k - kt * kGjTC;
    // the 16 lanes owning column k publish it and reduce their best unused row
    if (tx == kt) {
      double bv = -1.0;
      int bi = kGjMax;
#pragma unroll
      for (int r = 0; r < kGjTR; ++r) {
        double v = a[r][0];
#pragma unroll
        for (int c = 1; c < kGjTC; ++c) v = kc == c ? a[r][c] : v;
        S.col[b][r0 + r] = v;
        const double m = fabs(v) == fabs(v) ? fabs(v) : INFINITY;
        if (!((used >> r) & 1u) && m > bv) { bv = m; bi = r0 + r; }
      }
#pragma unroll
      for (int off = kGjGY / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, kGjGY);
        const int oi = __shfl_xor(bi, off, kGjGY);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (ty == 0) S.p[b] = bi;
    }
    __syncthreads();
    const int p = __builtin_amdgcn_readfirstlane(S.p[b]), pt = p / kGjTR, pr = p - pt * kGjTR;
    if (ty == pt) used |= 1u << pr;
    if (tid == 0) S.piv[k] = p;
    // the pivot row's entries in this lane's columns sit in lane pt of the
    // same 16-lane group
    double prow[kGjTC];
#pragma unroll
    for (int c = 0; c < kGjTC; ++c) prow[c] = 0.0;
#pragma unroll
    for (int r = 0; r < kGjTR; ++r)
      if (r == pr) {
#pragma unroll
        for (int c = 0; c < kGjTC; ++c) prow[c] = a[r][c];
      }
    const double inv = 1.0 / S.col[b][p];
    double pj[kGjTC];
#pragma unroll
    for (int c = 0; c < kGjTC; ++c) pj[c] = __shfl(prow[c], pt, kGjGY) * inv;
    // every element a[i][j] -= a[i][k] a[p][j] / d; then column k and row p
    // (whose values the uniform update does not produce) are overwritten
#pragma unroll
    for (int r = 0; r < kGjTR; ++r) {
      const double f = S.col[b][r0 + r];
#pragma unroll
      for (int c = 0; c < kGjTC; ++c) a[r][c] -= f * pj[c];
    }
    if (tx == kt) {
#pragma unroll
      for (int r = 0; r < kGjTR; ++r) {
        const double v = -S.col[b][r0 + r] * inv;
#pragma unroll
        for (int c = 0; c < kGjTC; ++c) a[r][c] = c == kc ? v : a[r][c];
      }
    }
    if (ty == pt) {
#pragma unroll
      for (int r = 0; r < kGjTR; ++r)
        if (r == pr) {
#pragma unroll
          for (int c = 0; c < kGjTC; ++c) a[r][c] = (tx == kt && c == kc) ? inv : pj[c];
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
