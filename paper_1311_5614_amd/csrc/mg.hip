// Multigrid level kernels on gfx950: operator apply / residual, box
// relaxation phases, transfers, right-hand side and interpolation.
//
// Paper references: MAC stencils (Sec. 2.2), the eliminated implicit system
// (Sec. 2.3.2, Sec. 3 matrix form, unsteady form of Sec. 8), Algorithm 1
// steps (Sec. 3), transfer operators (Sec. 3.1), hybrid coarse operators
// (Sec. 3.2), box relaxation (Sec. 5) with big boxes (Sec. 6).
#include "common.h"
#include "kernels.h"

#include "level_ops.h"

// Workgroups are dispatched to the eight XCDs round-robin by id, and each XCD
// has its own L2.  Block b of n runs work item xcd_remap(b, n): XCD x gets the
// x-th contiguous share of the items (a band of rows or of box rows), so
// neighbouring items that share cache lines share an L2.  A bijection on
// [0, n).
__device__ inline int xcd_remap(int b, int n) {
  const int m = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * m + (x < r ? x : r) + k;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_residual(LevelView<T> L, const T* __restrict__ b, const T* __restrict__ w, T* __restrict__ r) {
  residual_body<T>(L, b, w, r, xcd_remap(blockIdx.x, gridDim.x));
}
template <typename T>
__global__ void __launch_bounds__(256)
k_ib_rows(LevelView<T> L, const T* __restrict__ w, T* __restrict__ out, int mode, int colour) {
  ib_rows_body<T>(L, w, out, mode, blockIdx.x, blockIdx.y, gridDim.x, colour);
}
template <typename T>
__global__ void __launch_bounds__(256)
k_res_ib(LevelView<T> L, const T* __restrict__ b, const T* __restrict__ w, T* __restrict__ r, int nres_blocks) {
  const int blk = blockIdx.x;
  res_ib_body<T>(L, b, w, r, nres_blocks, blk < nres_blocks ? xcd_remap(blk, nres_blocks) : blk,
                 (int)gridDim.x - nres_blocks);
}
// W waves per workgroup: several on the large levels (fewer workgroups to
// dispatch), one where the colour has too few boxes to fill the chip that way.
// Each wave takes B nper consecutive boxes of the colour, B at a time.
template <typename T, int NB, int W, int B = 1, bool F = false>
__global__ void __launch_bounds__(64 * W)
k_box(LevelView<T> L, const T* __restrict__ r, T* __restrict__ w, int colour, int cnt, int nper) {
  const int q = (xcd_remap(blockIdx.x, gridDim.x) * W + (int)(threadIdx.x >> 6)) * nper * B;
  if constexpr (W > 1 && B == 1) {
    // several one-box waves: the shared plain inverse goes to LDS once per
    // workgroup, before any wave leaves (every lane takes part in the barrier)
    constexpr int ND = 2 * NB * (NB + 1) + NB * NB;
    __shared__ T sinv[ND * ND];
    for (int e = threadIdx.x; e < ND * ND; e += 64 * W) sinv[e] = L.ainv_plain[e];
    __syncthreads();
    if (q < cnt) box_body_n<T, NB, W, B, F, true>(L, r, w, colour, q, nper, cnt, sinv);
  } else {
    if (q < cnt) box_body_n<T, NB, W, B, F>(L, r, w, colour, q, nper, cnt);
  }
}
template <typename T>
__global__ void __launch_bounds__(kBigBoxLanes)
k_box_big(LevelView<T> L, const T* __restrict__ r, T* __restrict__ w, int colour) {
  const int wg = xcd_remap(blockIdx.x, gridDim.x);   // the row blocks of a box stay on one XCD
  box_body_big<T>(L, r, w, colour, wg / kBigBoxRowBlocks, wg % kBigBoxRowBlocks);
}
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(int Nf, const T* __restrict__ rf, T* __restrict__ rc,
                                                  T* __restrict__ wz, const T* __restrict__ yf, int walls) {
  restrict_body<T>(Nf, rf, rc, wz, blockIdx.x, yf, walls);
}
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(int Nf, const T* __restrict__ ec, T* __restrict__ wf,
                                                     int walls) {
  prolong_body<T>(Nf, ec, wf, blockIdx.x, walls);
}
template <typename T, int NB>
__global__ void __launch_bounds__(1024) k_tail(TailArgs<T> A) {
  tail_body<T, NB>(A);
}

// ---------------------------------------------------------------- a4: right-hand side
// b = [(rho/dt) u^n + S_0 G + g_u; (rho/dt) v^n + S_0 G + g_v; 0].  The spread
// force at a face sums, in ascending point order, W_k(face) G_k / h^2 over
// the points binned to the face's box.  walls (the cavity of Sec. 4): wall
// faces get 0 (prescribed normal velocity), and the top row of u faces the
// lid's ghost term 2 mu g(x) / h^2, g(x) = (1 - cos 2 pi x) / 2.
__global__ void __launch_bounds__(256)
k_rhs(PointView P, double c, double inv_h2, const double* __restrict__ u, const double* __restrict__ v,
      const double* __restrict__ gu, const double* __restrict__ gv, const double* __restrict__ G,
      double* __restrict__ b, int walls, double mu) {
  const int N = P.N, NN = N * N, msk = N - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * NN) return;
  const int comp = idx / NN, rem = idx - comp * NN;
  if (comp == 2) { b[idx] = 0.0; return; }
  const int j = rem / N, i = rem - j * N;
  if (walls && (comp == 0 ? i : j) == 0) { b[idx] = 0.0; return; }
  double val = 0.0;
  const double* f0 = comp == 0 ? u : v;
  const double* g0 = comp == 0 ? gu : gv;
  if (f0) val = c * f0[rem];
  double sp = 0.0;
  if (P.M > 0 && G) {
    const int box = (j / P.n) * P.nb + (i / P.n);
    const int* org = P.org + comp * P.M * 2;
    const double* wb = P.wts + (size_t)comp * P.M * IBMG_PATCH;
    for (int q = P.box_start[box]; q < P.box_start[box + 1]; ++q) {
      const int k = P.box_list[q];
      const int di = (i - org[2 * k]) & msk, dj = (j - org[2 * k + 1]) & msk;
      if (di < 4 && dj < 4) sp += wb[k * IBMG_PATCH + dj * 4 + di] * G[2 * k + comp];
    }
  }
  val += sp * inv_h2;
  if (g0) val += g0[rem];
  if (walls && comp == 0 && j == N - 1) val += mu * (1.0 - cospi(2.0 * i / N)) * inv_h2;
  b[idx] = val;
}

// ---------------------------------------------------------------- a14: U = S^* u, X += dt U
__global__ void __launch_bounds__(256)
k_interp(PointView P, const double* __restrict__ u, const double* __restrict__ v,
         double* __restrict__ U, double* __restrict__ X, double dt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * P.M) return;
  const int comp = t / P.M, k = t - comp * P.M;
  const int N = P.N, msk = N - 1;
  const double* f = comp == 0 ? u : v;
  const int oi = P.org[2 * t], oj = P.org[2 * t + 1];
  const double* wc = P.wts + (size_t)t * IBMG_PATCH;
  double acc = 0.0;
  for (int e = 0; e < 16; ++e) acc += wc[e] * f[((oj + (e >> 2)) & msk) * N + ((oi + (e & 3)) & msk)];
  if (U) U[2 * k + comp] = acc;
  if (X) X[2 * k + comp] += dt * acc;
}

// ---------------------------------------------------------------- launchers
namespace ibmg {

template <typename T> void launch_residual(hipStream_t s, const LevelView<T>& L, const T* b, const T* w, T* r,
                                           bool ib) {
  k_residual<T><<<nblk(3 * (size_t)L.N * L.N), 256, 0, s>>>(L, b, w, r);
  if (ib) k_ib_rows<T><<<dim3(ib_blocks(L.rowhint), 2), 256, 0, s>>>(L, w, r, b ? 2 : 1, -1);
}
template <typename T> void launch_res(hipStream_t s, const LevelView<T>& L, const T* b, const T* w, T* r, bool ib) {
  const int nres = (int)nblk(3 * (size_t)L.N * L.N);
  const int nib = ib ? 2 * ib_blocks(L.rowhint) : 0;
  k_res_ib<T><<<nres + nib, 256, 0, s>>>(L, b, w, r, nres);
}
template <typename T> void launch_box(hipStream_t s, const LevelView<T>& L, const T* r, T* w, int colour, bool ib) {
  LevelView<T> V = L;
  if (!ib) V.ib_index = nullptr;
  const int cnt = colour_count(L.ncol, L.nb);
  if (L.n == 8) {
    k_box_big<T><<<cnt * kBigBoxRowBlocks, kBigBoxLanes, 0, s>>>(V, r, w, colour);
  } else if (cnt >= kBoxWavesMax * 512) {
    // B boxes at a time per wave on levels without elastic rows once the
    // colour has enough boxes for cnt / B waves to fill the chip (4x4 boxes at
    // 256^2, 2048 per colour: 4.9 us with B = 1, 11 us with B = 2; at 1024^2,
    // 32768 per colour: 33 us with B = 1, 24 us with B = 4).  Boxes with
    // elastic rows cluster along the structure, and a wave taking several of
    // them issues their inverse loads one box after another (the 1024^2
    // eight-ring workload ran 9 % slower with B = 4), so such levels keep one
    // box per wave.  Groups per wave: one up to kBoxWaveTarget groups, then as
    // many as keep about kBoxWaveTarget waves in the launch.
    const int B = (L.n == 4 && !ib && cnt >= kBoxGroupMin) ? 4 : 1;
    const int groups = (cnt + B - 1) / B;
    const int nper = (B > 1 && groups > kBoxWaveTarget) ? groups / kBoxWaveTarget : 1;
    const int waves = (groups + nper - 1) / nper;
    constexpr int W1 = kBoxWavesOne;
    const int grid = (waves + (B == 4 ? kBoxWavesMax : W1) - 1) / (B == 4 ? kBoxWavesMax : W1);
    if (L.n == 4) {
      if (B == 4) k_box<T, 4, kBoxWavesMax, 4><<<grid, 64 * kBoxWavesMax, 0, s>>>(V, r, w, colour, cnt, nper);
      else k_box<T, 4, W1><<<grid, 64 * W1, 0, s>>>(V, r, w, colour, cnt, nper);
    } else if (L.n == 2) k_box<T, 2, W1><<<grid, 64 * W1, 0, s>>>(V, r, w, colour, cnt, nper);
    else k_box<T, 1, W1><<<grid, 64 * W1, 0, s>>>(V, r, w, colour, cnt, nper);
  } else {
    if (L.n == 4) k_box<T, 4, 1><<<cnt, 64, 0, s>>>(V, r, w, colour, cnt, 1);
    else if (L.n == 2) k_box<T, 2, 1><<<cnt, 64, 0, s>>>(V, r, w, colour, cnt, 1);
    else k_box<T, 1, 1><<<cnt, 64, 0, s>>>(V, r, w, colour, cnt, 1);
  }
}
// A colour phase in one box launch (plus the elastic-row pass on levels with
// elastic rows): the boxes form their Stokes residuals themselves from b and
// the iterate (box_body_n with F).  For four colours and 2 x 2 or 4 x 4 boxes.
template <typename T> void launch_phase_fused(hipStream_t s, const LevelView<T>& L, const T* b, T* w, int colour,
                                              bool ib, bool ib_rows) {
  LevelView<T> V = L;
  if (ib && ib_rows && L.act) k_ib_rows<T><<<dim3(ib_blocks(L.rowhint), 2), 256, 0, s>>>(L, w, nullptr, 0, colour);
  if (!ib) V.ib_index = nullptr;
  const int cnt = colour_count(L.ncol, L.nb);
  if (cnt >= kBoxWavesMax * 512) {
    const int B = (L.n == 4 && !ib && cnt >= kBoxGroupMin) ? 4 : 1;
    const int groups = (cnt + B - 1) / B;
    const int nper = (B > 1 && groups > kBoxWaveTarget) ? groups / kBoxWaveTarget : 1;
    const int waves = (groups + nper - 1) / nper;
    constexpr int W1 = kBoxWavesOne;
    const int grid = (waves + (B == 4 ? kBoxWavesMax : W1) - 1) / (B == 4 ? kBoxWavesMax : W1);
    if (L.n == 4) {
      if (B == 4) k_box<T, 4, kBoxWavesMax, 4, true><<<grid, 64 * kBoxWavesMax, 0, s>>>(V, b, w, colour, cnt, nper);
      else k_box<T, 4, W1, 1, true><<<grid, 64 * W1, 0, s>>>(V, b, w, colour, cnt, nper);
    } else {
      k_box<T, 2, W1, 1, true><<<grid, 64 * W1, 0, s>>>(V, b, w, colour, cnt, nper);
    }
  } else {
    if (L.n == 4) k_box<T, 4, 1, 1, true><<<cnt, 64, 0, s>>>(V, b, w, colour, cnt, 1);
    else k_box<T, 2, 1, 1, true><<<cnt, 64, 0, s>>>(V, b, w, colour, cnt, 1);
  }
}
template <typename T> void launch_restrict(hipStream_t s, int Nf, const T* rf, T* rc, T* wc_zero, const T* yf,
                                           int walls) {
  k_restrict<T><<<nblk(3 * (size_t)(Nf / 2) * (Nf / 2)), 256, 0, s>>>(Nf, rf, rc, wc_zero, yf, walls);
}
template <typename T> void launch_prolong_add(hipStream_t s, int Nf, const T* ec, T* wf, int walls) {
  k_prolong_add<T><<<nblk(3 * (size_t)Nf * Nf), 256, 0, s>>>(Nf, ec, wf, walls);
}
template <typename T> int launch_tail(hipStream_t s, const LevelView<T>* views, int ls, int L, int nu1, int nu2,
                                      bool ib, int nr, const T* b_in, T* w_out, const double* cainv) {
  TailArgs<T> A;
  size_t lds = 0;
  for (int l = 0; l < L; ++l) {
    A.v[l] = views[l];
    if (!ib) A.v[l].ib_index = nullptr;
    if (l >= ls) lds += 9 * (size_t)views[l].N * views[l].N * sizeof(T);
  }
  lds += (size_t)views[0].ndof * views[0].ndof * sizeof(T);
  A.ls = ls; A.L = L; A.nu1 = nu1; A.nu2 = nu2; A.ib = ib ? 1 : 0; A.nr = nr;
  A.b_in = b_in; A.w_out = w_out; A.cainv = cainv;
  if (views[0].n == 4) k_tail<T, 4><<<1, 1024, lds, s>>>(A);
  else if (views[0].n == 2) k_tail<T, 2><<<1, 1024, lds, s>>>(A);
  else k_tail<T, 1><<<1, 1024, lds, s>>>(A);
  return 0;
}
// Enable the tail kernels' dynamic LDS (up to lds bytes); outside any capture.
int prepare_tail(size_t lds) {
  if (lds <= 65536) return 0;
  const void* f[6] = {(const void*)k_tail<double, 1>, (const void*)k_tail<double, 2>, (const void*)k_tail<double, 4>,
                      (const void*)k_tail<float, 1>,  (const void*)k_tail<float, 2>,  (const void*)k_tail<float, 4>};
  for (const void* k : f)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -1;
  return 0;
}

void launch_rhs(hipStream_t s, const PointView& P, double c, double inv_h2, const double* u, const double* v,
                const double* gu, const double* gv, const double* G, double* b, int walls, double mu) {
  k_rhs<<<nblk(3 * (size_t)P.N * P.N), 256, 0, s>>>(P, c, inv_h2, u, v, gu, gv, G, b, walls, mu);
}
void launch_interp(hipStream_t s, const PointView& P, const double* u, const double* v, double* U,
                   double* X, double dt) {
  if (P.M > 0) k_interp<<<nblk(2 * (size_t)P.M), 256, 0, s>>>(P, u, v, U, X, dt);
}

#define IBMG_INST(T)                                                                                    \
  template void launch_residual<T>(hipStream_t, const LevelView<T>&, const T*, const T*, T*, bool);     \
  template void launch_res<T>(hipStream_t, const LevelView<T>&, const T*, const T*, T*, bool);         \
  template void launch_box<T>(hipStream_t, const LevelView<T>&, const T*, T*, int, bool);             \
  template void launch_phase_fused<T>(hipStream_t, const LevelView<T>&, const T*, T*, int, bool, bool);  \
  template void launch_restrict<T>(hipStream_t, int, const T*, T*, T*, const T*, int);                            \
  template void launch_prolong_add<T>(hipStream_t, int, const T*, T*, int);                             \
  template int launch_tail<T>(hipStream_t, const LevelView<T>*, int, int, int, int, bool, int, const T*, T*,   \
                              const double*);
IBMG_INST(double)
IBMG_INST(float)
#undef IBMG_INST

}  // namespace ibmg
