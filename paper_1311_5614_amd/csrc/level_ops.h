// Device bodies of the multigrid level operations, shared by the per-problem
// kernels (mg.hip) and the batched kernels (batch.hip): both call the same
// code on the same data, so a batched run reproduces per-problem runs bit
// for bit.  Each body takes the index of its block within the launch of one
// problem explicitly.  Paper references: MAC stencils (Sec. 2.2), the
// eliminated implicit system (Sec. 2.3.2, Sec. 3, unsteady form of Sec. 8),
// Algorithm 1 (Sec. 3), transfers (Sec. 3.1), hybrid coarse operators
// (Sec. 3.2), box relaxation (Sec. 5-6).
#pragma once
#include "common.h"

// ---------------------------------------------------------------- a8: y = A w or r = b - A w
// Stokes part here; the elastic rows are added by an elastic-row pass
// afterwards (ib_rows_body), or formed beside it (res_ib_body).
template <typename T>
__device__ inline void residual_body(const LevelView<T>& L, const T* __restrict__ b, const T* __restrict__ w,
                                     T* __restrict__ r, int blk) {
  const int NN = L.N * L.N, lg = __builtin_ctz(L.N);
  const int idx = blk * 256 + threadIdx.x;
  if (idx >= 3 * NN) return;
  const int comp = idx >> (2 * lg), rem = idx & (NN - 1);
  const int j = rem >> lg, i = rem & (L.N - 1);
  const T y = stokes_row(L, w, comp, i, j);
  r[idx] = b ? b[idx] - y : y;
}

// ---------------------------------------------------------------- (M_l w) on the active rows
// Sixteen lanes per active row split its window entries in a fixed pattern
// and reduce with a fixed shuffle tree; lane 0 stores.  mode 0: yib[row] =
// (M w)_f (formed before each colour phase from the iterate at the start of
// the phase -- a window reaches past the next box of the same colour, so the
// phase kernel must not evaluate it while those boxes are being updated);
// mode 1: out[f] += (M w)_f; mode 2: out[f] -= (M w)_f.
// Lane dx + R of the 16 takes window column dx (lanes past 2R idle) and sums
// its 2R + 1 entries top to bottom; every load is issued before the first
// product, so a row costs one memory latency.
template <typename T, int R>
__device__ inline T ib_col(const T* __restrict__ c, const T* __restrict__ x, int N, int i, int j, int lane) {
  constexpr int W = 2 * R + 1;
  const int msk = N - 1;
  T acc = T(0);
  if (lane < W) {
    const int dx = lane - R, ic = (i + dx) & msk;
    T cv[W], xv[W];
#pragma unroll
    for (int t = 0; t < W; ++t) {
      cv[t] = c[(t - R + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
      xv[t] = x[((j + t - R) & msk) * N + ic];
    }
#pragma unroll
    for (int t = 0; t < W; ++t) acc += cv[t] * xv[t];
  }
  return acc;
}

template <typename T>
__device__ inline T ib_row(const LevelView<T>& L, const T* __restrict__ w, int comp, int row, int lane, int& f) {
  const int N = L.N, NN = N * N, lg = __builtin_ctz(N);
  f = L.rows[comp * L.maxact + row];
  const int j = f >> lg, i = f & (N - 1);
  const T* c = L.win + ((size_t)comp * L.maxact + row) * IBMG_WS;
  const T* x = w + (size_t)comp * NN;
  T acc;
  if (L.reach <= 3) acc = ib_col<T, 3>(c, x, N, i, j, lane);
  else if (L.reach == 4) acc = ib_col<T, 4>(c, x, N, i, j, lane);
  else acc = ib_col<T, 5>(c, x, N, i, j, lane);
  acc += __shfl_xor(acc, 8, 16);
  acc += __shfl_xor(acc, 4, 16);
  acc += __shfl_xor(acc, 2, 16);
  acc += __shfl_xor(acc, 1, 16);
  return acc;
}

// Rows of one component, nblk workgroups striding over the active rows (the
// count is read on the device, so a captured launch stays valid when the
// active set changes).  colour >= 0 (mode 0, levels with per-colour row
// lists): only the rows in boxes of that colour, the only ones its phase
// reads.
template <typename T>
__device__ inline void ib_rows_body(const LevelView<T>& L, const T* __restrict__ w, T* __restrict__ out, int mode,
                                    int blk, int comp, int nblk, int colour = -1) {
  const int lane = threadIdx.x & 15, NN = L.N * L.N;
  const bool sub = colour >= 0 && L.crow;
  const int* list = sub ? L.crow + (size_t)(colour * 2 + comp) * L.maxact : nullptr;
  const int nrows = min(sub ? L.ncrow[colour * 2 + comp] : L.nact[comp], L.maxact);
  for (int q = (blk * 256 + threadIdx.x) >> 4; q < nrows; q += nblk * 16) {   // uniform over 16 lanes
    const int row = sub ? list[q] : q;
    int f;
    const T acc = ib_row(L, w, comp, row, lane, f);
    if (lane != 0) continue;
    if (mode == 0) L.yib[(size_t)comp * NN + f] = acc;
    else if (mode == 1) out[(size_t)comp * NN + f] += acc;
    else out[(size_t)comp * NN + f] -= acc;
  }
}

// ---------------------------------------------------------------- a9: one colour phase
// A phase is two launches so that every box of the colour solves from the
// iterate at the start of the phase (the 5-point stencil of a box's edge
// unknowns, and every elastic window, reaches unknowns of other boxes of the
// same colour).  k_res_ib: r = b - (Stokes part of A) w on every unknown, and
// yib = (M_l w) on every active elastic row (16 lanes per row, fixed-order
// shuffle tree).  k_box: one 64-lane wave per box of the colour; lane r takes
// res = r - yib at local unknown r, z = A_box^{-1} res, w[box] += z.  Boxes
// of one colour share no unknowns, so the update is race-free.  Boxes that
// touch the structure use their own FP64 inverse with the residual promoted
// to FP64.  The same fused pass forms the residual before each restriction,
// which subtracts yib (restrict_body).
template <typename T>
__device__ inline void res_ib_body(const LevelView<T>& L, const T* __restrict__ b, const T* __restrict__ w,
                                   T* __restrict__ r, int nres_blocks, int blk, int nib) {
  const int N = L.N, NN = N * N, lg = __builtin_ctz(N);
  if (blk < nres_blocks) {
    const int idx = blk * 256 + threadIdx.x;
    if (idx >= 3 * NN) return;
    const int comp = idx >> (2 * lg), rem = idx & (NN - 1);
    const int j = rem >> lg, i = rem & (N - 1);
    r[idx] = b[idx] - stokes_row(L, w, comp, i, j);
    return;
  }
  // elastic rows of both components, nib workgroups striding over them
  const int lane = threadIdx.x & 15;
  const int n0 = min(L.nact[0], L.maxact), n1 = min(L.nact[1], L.maxact);
  for (int q = ((blk - nres_blocks) * 256 + (int)threadIdx.x) >> 4; q < n0 + n1; q += nib * 16) {
    const int comp = q < n0 ? 0 : 1, row = q - comp * n0;
    int f;
    const T acc = ib_row(L, w, comp, row, lane, f);
    if (lane == 0) L.yib[(size_t)comp * NN + f] = acc;
  }
}

// Boxes of the colour q0 .. q0 + B nper - 1 (below cnt) on one 64-lane wave,
// B at a time, box edge NB fixed at compile time; W waves per workgroup.
// Lane r owns local unknown r of each box.  The lane's column of the shared
// plain inverse is loaded once and serves every box the wave takes: one
// column per box would read 56 x 56 inverse entries from L2 per box, far more
// than the box's own data.  For each group of B boxes every global load the
// lane needs (residual, elastic term, iterate) is issued before the residual
// exchange, so the group costs one memory latency before its products (the
// inverse of a box with elastic rows follows after it).  The residuals are
// exchanged through B 64-entry LDS slots per wave: with one wave per
// workgroup a workgroup barrier orders them, with several each wave orders
// its own.  Each box's arithmetic does not depend on B or nper.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kBoxWavesMax = 4;          // waves per workgroup on the large levels, several boxes per wave
constexpr int kBoxWavesOne = 8;          // waves per workgroup on the large levels, one box per wave: the
                                         // shared inverse staged in LDS serves eight boxes, and with the
                                         // box products unrolled by eight (64 registers per lane) eight
                                         // waves per SIMD stay resident (1024^2 fused phase: 31.7 -> 24.8 us)
constexpr int kBoxWaveTarget = 16384;    // waves per launch beyond which a wave takes several groups of boxes
constexpr int kBoxGroupMin = 16384;      // boxes per colour from which a wave takes 4x4 boxes four at a time (levels without elastic rows)

// F (fused): r is the level's right-hand side b, and each lane forms the
// Stokes residual of its unknown itself, b - (Stokes part of A) w, from the
// iterate at the start of the phase -- the same expression the residual pass
// evaluates, so the result is bitwise that of the two-launch phase.  Valid
// only where no box of the colour reads an unknown another box of the colour
// writes: four colours ((bx mod 2, by mod 2)) and boxes of at least 2 x 2
// cells put two boxes' width between boxes of one colour, more than the
// one-cell reach of the stencil.  The elastic rows still come from the
// elastic-row pass before the phase (their windows reach farther).
//
// LI, sinv (one box per wave): the shared plain inverse staged in LDS by
// the whole workgroup (k_box does it before any wave starts), read from
// there by every box of every wave -- column c of lane r at sinv[c ND + r],
// the same values in the same order as the register column, so the result
// does not change; the waves then take `nper` boxes each.  Without it a
// one-box wave reads the whole inverse from L2 for its single box (25 KB in
// FP64 against the box's own 1.3 KB).
template <typename T, int NB, int W = 1, int B = 1, bool F = false, bool LI = false>
__device__ inline void box_body_n(const LevelView<T>& L, const T* __restrict__ r, T* __restrict__ w, int colour,
                                  int q0, int nper = 1, int cnt = 0x7fffffff, const T* sinv = nullptr) {
  constexpr int ND = 2 * NB * (NB + 1) + NB * NB;
  __shared__ double res_all[W][B][64];
  double (*res)[64] = res_all[W == 1 ? 0 : threadIdx.x >> 6];
  const int lane = threadIdx.x & 63, N = L.N, NN = N * N;
  // the lane's column of the shared plain inverse, kept in registers for
  // every box the wave takes.  One box per wave: loaded after the box's own
  // loads, so that the residual exchange does not wait for it; several:
  // loaded first (fewer registers live across the loop)
  T a[ND];
  if constexpr (B > 1) {
    if (lane < ND) {
#pragma unroll
      for (int c = 0; c < ND; ++c) a[c] = L.ainv_plain[c * ND + lane];
    }
  }
  // one box per wave comes with one group per wave unless the inverse is in
  // LDS: a compile-time single pass leaves the column dead on the path of
  // boxes with elastic rows, whose inverse loads then all issue together
  const int np = (B == 1 && !LI) ? 1 : nper;
  for (int k = 0; k < np; ++k) {
    const int qb = q0 + k * B;
    if (qb >= cnt) break;   // uniform over the wave
    int ibx[B];
    size_t g[B];
    T y[B], wv[B], yb[B];
    int comp = 0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      ibx[b] = -2;   // past the colour's last box
      g[b] = 0;
      y[b] = T(0);
      wv[b] = T(0);
      yb[b] = T(0);
      if (qb + b >= cnt) continue;
      int bx, by;
      colour_box(qb + b, colour, L.ncol, L.nb, bx, by);
      ibx[b] = L.ib_index ? L.ib_index[by * L.nb + bx] : -1;
      if (lane < ND) {
        int i, j;
        box_dof(lane, bx, by, NB, N, comp, i, j);
        g[b] = (size_t)comp * NN + (size_t)j * N + i;
        if constexpr (F) y[b] = r[g[b]] - stokes_row(L, w, comp, i, j);
        else y[b] = r[g[b]];
        wv[b] = w[g[b]];
        // zero off the active rows.  One box per wave: loaded whatever the
        // box's class, so that no load waits for another (the launch is
        // latency-bound); several: only for boxes with elastic rows (fewer
        // registers; the launch is bandwidth-bound)
        if constexpr (B == 1) {
          if (L.yib && comp < 2) yb[b] = L.yib[g[b]];
        } else {
          if (ibx[b] >= 0 && L.yib && comp < 2) yb[b] = L.yib[g[b]];
        }
      }
    }
    if (B == 1 && !LI && k == 0 && lane < ND) {
#pragma unroll
      for (int c = 0; c < ND; ++c) a[c] = L.ainv_plain[c * ND + lane];
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (ibx[b] >= 0 && comp < 2) y[b] -= yb[b];
    if (k > 0) {   // the previous boxes' products have read the slots
      if constexpr (W == 1) __syncthreads();
      else wave_sync();
    }
    if (lane < ND) {
#pragma unroll
      for (int b = 0; b < B; ++b) res[b][lane] = (double)y[b];
    }
    if constexpr (W == 1) __syncthreads();
    else wave_sync();
    if (lane < ND) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (ibx[b] == -2) continue;
        if (ibx[b] >= 0) {
          const double* A = L.ainv_ib + (size_t)ibx[b] * ND * ND;
          double z = 0.0;
          if constexpr (B == 1) {
            // one box per wave: unrolled by eight, not fully (the register
            // pressure of 56 loads in flight would halve the waves resident
            // per SIMD)
#pragma unroll 8
            for (int c = 0; c < ND; ++c) z += A[c * ND + lane] * res[b][c];
          } else {
#pragma unroll
            for (int c = 0; c < ND; ++c) z += A[c * ND + lane] * res[b][c];
          }
          w[g[b]] = wv[b] + L.omega * (T)z;
        } else if constexpr (LI) {
          T z = T(0);
#pragma unroll 8
          for (int c = 0; c < ND; ++c) z += sinv[c * ND + lane] * (T)res[b][c];
          w[g[b]] = wv[b] + L.omega * z;
        } else {
          T z = T(0);
#pragma unroll
          for (int c = 0; c < ND; ++c) z += a[c] * (T)res[b][c];
          w[g[b]] = wv[b] + L.omega * z;
        }
      }
    }
  }
}

// Boxes of 8 x 8 cells (208 unknowns): four 256-lane workgroups per box, each
// computing 52 rows of z = A_box^{-1} res, so that the inverse (173 KB FP32
// shared, 346 KB FP64 per box with elastic rows) is read by four CUs.  In a
// workgroup, wave q takes columns 52 q .. 52 q + 51 of its rows (one row per
// lane, loaded before the barrier like box_body_n's single column; the box's
// class is known first, so only the inverse it uses is loaded) and the four
// partial sums are added in a fixed order.  Boxes of one colour share no
// unknowns, and every workgroup reads only r and the elastic term and writes
// only its own rows of w, so the workgroups of a box need no ordering.
constexpr int kBigBoxLanes = 256, kBigBoxRowBlocks = 4;

template <typename T, typename A>
__device__ inline void big_box_rows(const A* __restrict__ inv, T y, int row, int rr, int q, bool act, size_t gr,
                                    T wv, T* __restrict__ w, double* res, double (*part)[52], T omega) {
  constexpr int ND = 208, CP = 52;
  A a[CP];
  if (act) {
#pragma unroll
    for (int c = 0; c < CP; ++c) a[c] = inv[(q * CP + c) * ND + row];
  }
  if (threadIdx.x < ND) res[threadIdx.x] = (double)y;
  __syncthreads();
  if (act) {
    A z = A(0);
#pragma unroll
    for (int c = 0; c < CP; ++c) z += a[c] * (A)res[q * CP + c];
    part[q][rr] = (double)z;
  }
  __syncthreads();
  if (act && q == 0) {
    const A z = (((A)part[0][rr] + (A)part[1][rr]) + (A)part[2][rr]) + (A)part[3][rr];
    w[gr] = wv + omega * (T)z;
  }
}

template <typename T>
__device__ inline void box_body_big(const LevelView<T>& L, const T* __restrict__ r, T* __restrict__ w, int colour,
                                    int blk, int rb) {
  constexpr int NB = 8, ND = 2 * NB * (NB + 1) + NB * NB, RR = ND / kBigBoxRowBlocks, PARTS = 4;
  static_assert(RR == 52 && ND / PARTS == 52, "8 x 8 box split");
  __shared__ double res[ND];
  __shared__ double part[PARTS][RR];
  int bx, by;
  colour_box(blk, colour, L.ncol, L.nb, bx, by);
  const int lane = threadIdx.x, N = L.N, NN = N * N;
  const int ibx = L.ib_index ? L.ib_index[by * L.nb + bx] : -1;
  // the residual of the whole box
  T y = T(0), yb = T(0);
  int comp = 0;
  if (lane < ND) {
    int i, j;
    box_dof(lane, bx, by, NB, N, comp, i, j);
    const size_t g = (size_t)comp * NN + (size_t)j * N + i;
    y = r[g];
    if (L.yib && comp < 2) yb = L.yib[g];   // zero off the active rows
  }
  // this workgroup's rows: lane = 64 q + rr, row = RR rb + rr
  const int rr = lane & 63, q = lane >> 6, row = rb * RR + rr;
  const bool act = rr < RR;
  size_t gr = 0;
  T wv = T(0);
  if (act) {
    int c2, i2, j2;
    box_dof(row, bx, by, NB, N, c2, i2, j2);
    gr = (size_t)c2 * NN + (size_t)j2 * N + i2;
    if (q == 0) wv = w[gr];
  }
  if (ibx >= 0) {
    if (comp < 2) y -= yb;
    big_box_rows<T, double>(L.ainv_ib + (size_t)ibx * ND * ND, y, row, rr, q, act, gr, wv, w, res, part, L.omega);
  } else {
    big_box_rows<T, T>(L.ainv_plain, y, row, rr, q, act, gr, wv, w, res, part, L.omega);
  }
}

// Boxes of 1, 2 or 4 cells (8 x 8 boxes go through box_body_big).
template <typename T>
__device__ inline void box_body(const LevelView<T>& L, const T* __restrict__ r, T* __restrict__ w, int colour,
                                int blk) {
  if (L.n == 4) box_body_n<T, 4>(L, r, w, colour, blk);
  else if (L.n == 2) box_body_n<T, 2>(L, r, w, colour, blk);
  else box_body_n<T, 1>(L, r, w, colour, blk);
}

// ---------------------------------------------------------------- a10: restriction (Sec. 3.1)
// The coarse correction of Algorithm 1 starts from zero, so the same launch
// clears the coarse iterate (wz, nullable).  yf (nullable): the elastic term
// of the fine residual, zero off the active rows -- the fine residual is
// rf - yf, formed here (one subtraction, as the elastic-row pass would).
template <typename T>
__device__ inline T res_at(const T* __restrict__ rf, const T* __restrict__ yf, size_t i) {
  return yf ? rf[i] - yf[i] : rf[i];
}

// walls: the coarse wall faces (u: I = 0, v: J = 0) restrict to zero; the
// other coarse faces read only interior fine faces.
template <typename T>
__device__ inline void restrict_body(int Nf, const T* __restrict__ rf, T* __restrict__ rc, T* __restrict__ wz,
                                     int blk, const T* __restrict__ yf = nullptr, int walls = 0) {
  const int Nc = Nf / 2, NNc = Nc * Nc, NNf = Nf * Nf, mf = Nf - 1, lgc = __builtin_ctz(Nc);
  const int idx = blk * 256 + threadIdx.x;
  if (idx >= 3 * NNc) return;
  const int comp = idx >> (2 * lgc), rem = idx & (NNc - 1);
  const int J = rem >> lgc, I = rem & (Nc - 1);
  const T* f = rf + (size_t)comp * NNf;
  const T* y = yf && comp < 2 ? yf + (size_t)comp * NNf : nullptr;
  T s = T(0);
  if (comp == 0) {
    for (int e = 0; e < 2; ++e) {
      const int jj = 2 * J + e;
      s += T(0.125) * res_at(f, y, jj * Nf + ((2 * I - 1) & mf)) + T(0.25) * res_at(f, y, jj * Nf + 2 * I) +
           T(0.125) * res_at(f, y, jj * Nf + ((2 * I + 1) & mf));
    }
  } else if (comp == 1) {
    for (int e = 0; e < 2; ++e) {
      const int ii = 2 * I + e;
      s += T(0.125) * res_at(f, y, ((2 * J - 1) & mf) * Nf + ii) + T(0.25) * res_at(f, y, (2 * J) * Nf + ii) +
           T(0.125) * res_at(f, y, ((2 * J + 1) & mf) * Nf + ii);
    }
  } else {
    s = T(0.25) * (f[2 * J * Nf + 2 * I] + f[2 * J * Nf + 2 * I + 1] + f[(2 * J + 1) * Nf + 2 * I] +
                   f[(2 * J + 1) * Nf + 2 * I + 1]);
  }
  if (walls && ((comp == 0 && I == 0) || (comp == 1 && J == 0))) s = T(0);
  rc[idx] = s;
  if (wz) wz[idx] = T(0);
}

// ---------------------------------------------------------------- a11: prolong and correct (Sec. 3.1)
template <typename T>
__device__ inline T bilinear(const T* c, int Nc, int in, int it, bool normal_is_x) {
  // in: fine index along the face normal, it: along the tangent
  const int mc = Nc - 1;
  int n0, n1;
  T wn0, wn1;
  if ((in & 1) == 0) { n0 = in >> 1; n1 = n0; wn0 = T(1); wn1 = T(0); }
  else { n0 = (in - 1) >> 1; n1 = ((in + 1) >> 1) & mc; wn0 = T(0.5); wn1 = T(0.5); }
  const int t0 = it >> 1;
  const int t1 = ((it & 1) == 0 ? t0 - 1 : t0 + 1) & mc;
  auto at = [&](int a, int b) -> T { return normal_is_x ? c[b * Nc + a] : c[a * Nc + b]; };
  T s = T(0.75) * (wn0 * at(n0, t0)) + T(0.25) * (wn0 * at(n0, t1));
  if ((in & 1) != 0) s += T(0.75) * (wn1 * at(n1, t0)) + T(0.25) * (wn1 * at(n1, t1));
  return s;
}

// Bilinear prolongation with walls: coarse wall faces (normal index 0; Nc
// stands for the wall at the far side) contribute nothing, and across a
// wall parallel to the face the coarse field's ghost is -e, so the fine row
// next to the wall takes 3/4 - 1/4 = 1/2 of its coarse row.  Fine wall faces
// get nothing.
template <typename T>
__device__ inline T bilinear_walls(const T* c, int Nc, int in, int it, bool normal_is_x) {
  if (in == 0) return T(0);
  auto at = [&](int a, int b) -> T { return normal_is_x ? c[b * Nc + a] : c[a * Nc + b]; };
  const int t0 = it >> 1;
  const int t1 = (it & 1) == 0 ? t0 - 1 : t0 + 1;
  const bool t1in = t1 >= 0 && t1 < Nc;
  auto tang = [&](int n) -> T {   // the tangential pair of coarse normal index n
    return t1in ? T(0.75) * at(n, t0) + T(0.25) * at(n, t1) : T(0.5) * at(n, t0);
  };
  if ((in & 1) == 0) return tang(in >> 1);
  const int n0 = (in - 1) >> 1, n1 = (in + 1) >> 1;
  T s = T(0);
  if (n0 > 0) s += T(0.5) * tang(n0);
  if (n1 < Nc) s += T(0.5) * tang(n1);
  return s;
}

template <typename T>
__device__ inline void prolong_body(int Nf, const T* __restrict__ ec, T* __restrict__ wf, int blk, int walls = 0) {
  const int Nc = Nf / 2, NNc = Nc * Nc, NNf = Nf * Nf, lgf = __builtin_ctz(Nf);
  const int idx = blk * 256 + threadIdx.x;
  if (idx >= 3 * NNf) return;
  const int comp = idx >> (2 * lgf), rem = idx & (NNf - 1);
  const int j = rem >> lgf, i = rem & (Nf - 1);
  const T* c = ec + (size_t)comp * NNc;
  T add;
  if (comp == 0) add = walls ? bilinear_walls(c, Nc, i, j, true) : bilinear(c, Nc, i, j, true);
  else if (comp == 1) add = walls ? bilinear_walls(c, Nc, j, i, false) : bilinear(c, Nc, j, i, false);
  else add = c[(j >> 1) * Nc + (i >> 1)];
  wf[idx] += add;
}

// ---------------------------------------------------------------- small levels in one workgroup
// Levels of at most 32 x 32 cells carry too little work to fill the chip; one
// 1024-thread workgroup runs all of their colour phases (k_tail) with
// workgroup barriers in place of kernel launches.  Same arithmetic as k_res_ib and
// k_box: the residual and the elastic rows are formed before each colour
// from the iterate at its start, then each wave solves one box of the colour
// per round, in the same fixed order as k_box.
// One thread per elastic row, window loops unrolled so that all loads of a
// window row are in flight together (fixed summation order: dy, then dx).
template <typename T, int R>
__device__ inline T win_row(const T* __restrict__ c, const T* __restrict__ x, int N, int i, int j) {
  const int msk = N - 1;
  T acc = T(0);
#pragma unroll
  for (int dy = -R; dy <= R; ++dy) {
    const T* row = x + ((j + dy) & msk) * N;
    const T* cw = c + (dy + IBMG_WR) * IBMG_WW + IBMG_WR;
#pragma unroll
    for (int dx = -R; dx <= R; ++dx) acc += cw[dx] * row[(i + dx) & msk];
  }
  return acc;
}

template <typename T>
__device__ void small_ib_rows(const LevelView<T>& L, const T* __restrict__ w, T* __restrict__ out, int mode) {
  const int N = L.N, NN = N * N;
  const int n0 = min(L.nact[0], L.maxact), n1 = min(L.nact[1], L.maxact);
  for (int q = threadIdx.x; q < n0 + n1; q += blockDim.x) {
    const int comp = q < n0 ? 0 : 1, row = q - comp * n0;
    const int f = L.rows[comp * L.maxact + row];
    const int j = f / N, i = f - j * N;
    const T* c = L.win + ((size_t)comp * L.maxact + row) * IBMG_WS;
    const T* x = w + (size_t)comp * NN;
    T acc;
    if (L.reach <= 3) acc = win_row<T, 3>(c, x, N, i, j);
    else if (L.reach == 4) acc = win_row<T, 4>(c, x, N, i, j);
    else acc = win_row<T, 5>(c, x, N, i, j);
    if (mode == 0) L.yib[(size_t)comp * NN + f] = acc;
    else if (mode == 1) out[(size_t)comp * NN + f] += acc;
    else out[(size_t)comp * NN + f] -= acc;
  }
}

// Ap: the level's plain-box inverse staged in LDS.  The box edge NB is a
// compile-time constant so that every inverse load of a box solve is issued
// before the first product needs it.
template <typename T, int NB>
__device__ void small_sweep(const LevelView<T>& L, const T* __restrict__ b, T* __restrict__ w, T* __restrict__ r,
                            bool ib, const T* __restrict__ Ap) {
  __shared__ double res[16][64];
  constexpr int nd = 2 * NB * (NB + 1) + NB * NB;
  const int N = L.N, NN = N * N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  for (int colour = 0; colour < L.ncol; ++colour) {
    // residual and elastic rows from the iterate at the start of the colour
    for (int idx = threadIdx.x; idx < 3 * NN; idx += blockDim.x) {
      const int comp = idx / NN, rem = idx - comp * NN;
      const int j = rem / N, i = rem - j * N;
      r[idx] = b[idx] - stokes_row(L, w, comp, i, j);
    }
    if (ib) small_ib_rows<T>(L, w, nullptr, 0);
    __syncthreads();
    const int cnt = colour_count(L.ncol, L.nb);
    const int rounds = (cnt + nwaves - 1) / nwaves;
    for (int round = 0; round < rounds; ++round) {
      const int q = round * nwaves + wave;
      const bool active = q < cnt;
      int bx = 0, by = 0, comp = 0, i = 0, j = 0, ibx = -1;
      size_t g = 0;
      if (active) {
        colour_box(q, colour, L.ncol, L.nb, bx, by);
        ibx = ib ? L.ib_index[by * L.nb + bx] : -1;
        if (lane < nd) {
          box_dof(lane, bx, by, NB, N, comp, i, j);
          g = (size_t)comp * NN + (size_t)j * N + i;
          T y = r[g];
          if (ibx >= 0 && comp < 2 && L.yib) y -= L.yib[g];   // zero off the active rows
          res[wave][lane] = (double)y;
        }
      }
      __syncthreads();
      if (active && lane < nd) {
        if (ibx >= 0) {
          const double* A = L.ainv_ib + (size_t)ibx * nd * nd;
          double z = 0.0;
#pragma unroll
          for (int c = 0; c < nd; ++c) z += A[c * nd + lane] * res[wave][c];
          w[g] += L.omega * (T)z;
        } else {
          T z = T(0);
#pragma unroll 8
          for (int c = 0; c < nd; ++c) z += Ap[c * nd + lane] * (T)res[wave][c];
          w[g] += L.omega * z;
        }
      }
      __syncthreads();
    }
  }
}

// The tail of the V-cycle: every level from ls down to the coarsest, and the
// coarsest exact solve, in one workgroup with the fields of those levels
// resident in LDS.  Entry: b_ls in global memory (the restricted residual of
// the level above, or the preconditioner input when ls = 0).  Exit: w_ls in
// global memory.  Same steps as the per-level kernels (Algorithm 1).
// Dynamic LDS of the tail: w, b, r of every level from ls down (9 N_l^2
// values), then one plain-box inverse (nd^2 values).
template <typename T>
struct TailArgs {
  LevelView<T> v[IBMG_MAX_LEVELS];
  int ls, L, nu1, nu2, ib, nr;
  const T* b_in;
  T* w_out;
  const double* cainv;
};

template <typename T>
__device__ void tail_restrict(int N, const T* __restrict__ r, T* __restrict__ bc, T* __restrict__ wc) {
  const int NN = N * N, Nc = N / 2, NNc = Nc * Nc, mf = N - 1;
  for (int idx = threadIdx.x; idx < 3 * NNc; idx += blockDim.x) {
    const int comp = idx / NNc, rem = idx - comp * NNc;
    const int J = rem / Nc, I = rem - J * Nc;
    const T* f = r + (size_t)comp * NN;
    T sacc = T(0);
    if (comp == 0) {
      for (int e = 0; e < 2; ++e) {
        const int jj = 2 * J + e;
        sacc += T(0.125) * f[jj * N + ((2 * I - 1) & mf)] + T(0.25) * f[jj * N + 2 * I] +
                T(0.125) * f[jj * N + ((2 * I + 1) & mf)];
      }
    } else if (comp == 1) {
      for (int e = 0; e < 2; ++e) {
        const int ii = 2 * I + e;
        sacc += T(0.125) * f[((2 * J - 1) & mf) * N + ii] + T(0.25) * f[(2 * J) * N + ii] +
                T(0.125) * f[((2 * J + 1) & mf) * N + ii];
      }
    } else {
      sacc = T(0.25) * (f[2 * J * N + 2 * I] + f[2 * J * N + 2 * I + 1] + f[(2 * J + 1) * N + 2 * I] +
                        f[(2 * J + 1) * N + 2 * I + 1]);
    }
    bc[idx] = sacc;
    wc[idx] = T(0);
  }
}

// Copy level l's plain-box inverse into the LDS slot Ap.
template <typename T, int NB>
__device__ inline void stage_plain(const LevelView<T>& L, T* __restrict__ Ap) {
  constexpr int nd = 2 * NB * (NB + 1) + NB * NB;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) Ap[idx] = L.ainv_plain[idx];
  __syncthreads();
}

template <typename T, int NB>
__device__ inline void tail_body(const TailArgs<T>& A) {
  extern __shared__ double smem[];
  T* w[IBMG_MAX_LEVELS];
  T* b[IBMG_MAX_LEVELS];
  T* r[IBMG_MAX_LEVELS];
  T* Ap;
  {
    T* p = reinterpret_cast<T*>(smem);
    for (int l = A.ls; l < A.L; ++l) {
      const int n3 = 3 * A.v[l].N * A.v[l].N;
      w[l] = p; p += n3;
      b[l] = p; p += n3;
      r[l] = p; p += n3;
    }
    Ap = p;
  }
  const int ib = A.ib;
  {
    const int n3 = 3 * A.v[A.ls].N * A.v[A.ls].N;
    for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) {
      b[A.ls][idx] = A.b_in[idx];
      w[A.ls][idx] = T(0);
    }
  }
  __syncthreads();
  for (int l = A.ls; l + 1 < A.L; ++l) {
    const LevelView<T>& L = A.v[l];
    const int N = L.N, NN = N * N;
    if (A.nu1 > 0) stage_plain<T, NB>(L, Ap);
    for (int s = 0; s < A.nu1; ++s) small_sweep<T, NB>(L, b[l], w[l], r[l], ib != 0, Ap);
    for (int idx = threadIdx.x; idx < 3 * NN; idx += blockDim.x) {
      const int comp = idx / NN, rem = idx - comp * NN;
      const int j = rem / N, i = rem - j * N;
      r[l][idx] = b[l][idx] - stokes_row(L, w[l], comp, i, j);
    }
    __syncthreads();
    if (ib) small_ib_rows<T>(L, w[l], r[l], 2);
    __syncthreads();
    tail_restrict<T>(N, r[l], b[l + 1], w[l + 1]);
    __syncthreads();
  }
  {
    // coarsest: w = first nr-1 entries of A^{-1} [b; 0]; one wave per row
    const int lc = A.L - 1, nr = A.nr;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    for (int row = wave; row < nr - 1; row += nwaves) {
      const double* a = A.cainv + (size_t)row * nr;
      double acc = 0.0;
      for (int c = lane; c < nr - 1; c += 64) acc += a[c] * (double)b[lc][c];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
      if (lane == 0) w[lc][row] = (T)acc;
    }
    __syncthreads();
  }
  for (int l = A.L - 2; l >= A.ls; --l) {
    const LevelView<T>& L = A.v[l];
    const int N = L.N, NN = N * N, Nc = N / 2, NNc = Nc * Nc;
    for (int idx = threadIdx.x; idx < 3 * NN; idx += blockDim.x) {
      const int comp = idx / NN, rem = idx - comp * NN;
      const int j = rem / N, i = rem - j * N;
      const T* c = w[l + 1] + (size_t)comp * NNc;
      T add;
      if (comp == 0) add = bilinear(c, Nc, i, j, true);
      else if (comp == 1) add = bilinear(c, Nc, j, i, false);
      else add = c[(j >> 1) * Nc + (i >> 1)];
      w[l][idx] += add;
    }
    __syncthreads();
    if (A.nu2 > 0) stage_plain<T, NB>(L, Ap);
    for (int s = 0; s < A.nu2; ++s) small_sweep<T, NB>(L, b[l], w[l], r[l], ib != 0, Ap);
  }
  {
    const int n3 = 3 * A.v[A.ls].N * A.v[A.ls].N;
    for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) A.w_out[idx] = w[A.ls][idx];
  }
}


template <typename T>
__device__ inline void tail_body_n(const TailArgs<T>& A) {
  const int n = A.v[A.ls].n;
  if (n == 4) tail_body<T, 4>(A);
  else if (n == 2) tail_body<T, 2>(A);
  else tail_body<T, 1>(A);   // n = 1; with 8 x 8 boxes the tail is the coarsest level alone (no box)
}
