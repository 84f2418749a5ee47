// Multigrid level kernels on gfx950: operator apply / residual, box
// relaxation phases, transfers, right-hand side and interpolation.
//
// Paper references: MAC stencils (Sec. 2.2), the eliminated implicit system
// (Sec. 2.3.2, Sec. 3 matrix form, unsteady form of Sec. 8), Algorithm 1
// steps (Sec. 3), transfer operators (Sec. 3.1), hybrid coarse operators
// (Sec. 3.2), box relaxation (Sec. 5) with big boxes (Sec. 6).
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------- t = C_l w
template <typename T>
__global__ void __launch_bounds__(256) k_gather(LevelView<T> L, const T* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * L.M) return;
  const int comp = t / L.M;
  const int N = L.N, msk = N - 1;
  const T* f = w + (size_t)comp * N * N;
  const int oi = L.orgC[2 * t], oj = L.orgC[2 * t + 1];
  const T* wc = L.wC + (size_t)t * IBMG_PATCH;
  T acc = T(0);
#pragma unroll
  for (int e = 0; e < 16; ++e) acc += wc[e] * f[((oj + (e >> 2)) & msk) * N + ((oi + (e & 3)) & msk)];
  L.t[t] = acc;
}

// ---------------------------------------------------------------- a8: y = A w or r = b - A w
template <typename T>
__global__ void __launch_bounds__(256)
k_residual(LevelView<T> L, const T* __restrict__ b, const T* __restrict__ w, T* __restrict__ r, int ib) {
  const int NN = L.N * L.N;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * NN) return;
  const int comp = idx / NN, rem = idx - comp * NN;
  const int j = rem / L.N, i = rem - j * L.N;
  T y = stokes_row(L, w, comp, i, j);
  if (ib && comp < 2) y += ib_face(L, comp, i, j);
  r[idx] = b ? b[idx] - y : y;
}

// ---------------------------------------------------------------- a9: one colour phase
// One 64-lane workgroup per box of colour (cx, cy).  Lane r forms the
// residual of local unknown r from the values at the start of the phase,
// then z = A_box^{-1} res and w[box] += z.  Boxes of one colour share no
// unknowns, so the in-place update is race-free.  Boxes that touch the
// structure use their own FP64 inverse with the residual promoted to FP64.
template <typename T>
__global__ void __launch_bounds__(64)
k_phase(LevelView<T> L, const T* __restrict__ b, T* __restrict__ w, int cx, int cy) {
  __shared__ double res[64];
  const int half = L.nb / 2;
  const int q = blockIdx.x;
  const int bx = 2 * (q % half) + cx, by = 2 * (q / half) + cy;
  const int box = by * L.nb + bx;
  const int r = threadIdx.x, nd = L.ndof, N = L.N, NN = N * N;
  const int ibx = L.ib_index ? L.ib_index[box] : -1;
  int comp = 0, i = 0, j = 0;
  size_t g = 0;
  if (r < nd) {
    box_dof(r, bx, by, L.n, N, comp, i, j);
    g = (size_t)comp * NN + (size_t)j * N + i;
    T y = stokes_row(L, w, comp, i, j);
    if (ibx >= 0 && comp < 2) y += ib_face(L, comp, i, j);
    res[r] = (double)(b[g] - y);
  }
  __syncthreads();
  if (r >= nd) return;
  if (ibx >= 0) {
    const double* A = L.ainv_ib + (size_t)ibx * nd * nd;
    double z = 0.0;
    for (int c = 0; c < nd; ++c) z += A[c * nd + r] * res[c];
    w[g] += (T)z;
  } else {
    const T* A = L.ainv_plain;
    T z = T(0);
    for (int c = 0; c < nd; ++c) z += A[c * nd + r] * (T)res[c];
    w[g] += z;
  }
}

// ---------------------------------------------------------------- a10: restriction (Sec. 3.1)
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(int Nf, const T* __restrict__ rf, T* __restrict__ rc) {
  const int Nc = Nf / 2, NNc = Nc * Nc, NNf = Nf * Nf, mf = Nf - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * NNc) return;
  const int comp = idx / NNc, rem = idx - comp * NNc;
  const int J = rem / Nc, I = rem - J * Nc;
  const T* f = rf + (size_t)comp * NNf;
  T s = T(0);
  if (comp == 0) {
    for (int e = 0; e < 2; ++e) {
      const int jj = 2 * J + e;
      s += T(0.125) * f[jj * Nf + ((2 * I - 1) & mf)] + T(0.25) * f[jj * Nf + 2 * I] +
           T(0.125) * f[jj * Nf + ((2 * I + 1) & mf)];
    }
  } else if (comp == 1) {
    for (int e = 0; e < 2; ++e) {
      const int ii = 2 * I + e;
      s += T(0.125) * f[((2 * J - 1) & mf) * Nf + ii] + T(0.25) * f[(2 * J) * Nf + ii] +
           T(0.125) * f[((2 * J + 1) & mf) * Nf + ii];
    }
  } else {
    s = T(0.25) * (f[2 * J * Nf + 2 * I] + f[2 * J * Nf + 2 * I + 1] + f[(2 * J + 1) * Nf + 2 * I] +
                   f[(2 * J + 1) * Nf + 2 * I + 1]);
  }
  rc[idx] = s;
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

template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(int Nf, const T* __restrict__ ec, T* __restrict__ wf) {
  const int Nc = Nf / 2, NNc = Nc * Nc, NNf = Nf * Nf;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * NNf) return;
  const int comp = idx / NNf, rem = idx - comp * NNf;
  const int j = rem / Nf, i = rem - j * Nf;
  const T* c = ec + (size_t)comp * NNc;
  T add;
  if (comp == 0) add = bilinear(c, Nc, i, j, true);
  else if (comp == 1) add = bilinear(c, Nc, j, i, false);
  else add = c[(j >> 1) * Nc + (i >> 1)];
  wf[idx] += add;
}

// ---------------------------------------------------------------- a4: right-hand side
// b = [(rho/dt) u^n + S_0 G + g_u; (rho/dt) v^n + S_0 G + g_v; 0].  The spread
// force at a face sums, in ascending point order, W_k(face) G_k / h^2 over
// the points binned to the face's box.
__global__ void __launch_bounds__(256)
k_rhs(LevelView<double> L, double inv_h2, const double* __restrict__ u, const double* __restrict__ v,
      const double* __restrict__ gu, const double* __restrict__ gv, const double* __restrict__ G,
      double* __restrict__ b) {
  const int N = L.N, NN = N * N, msk = N - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * NN) return;
  const int comp = idx / NN, rem = idx - comp * NN;
  if (comp == 2) { b[idx] = 0.0; return; }
  const int j = rem / N, i = rem - j * N;
  double val = 0.0;
  const double* f0 = comp == 0 ? u : v;
  const double* g0 = comp == 0 ? gu : gv;
  if (f0) val = L.c * f0[rem];
  double sp = 0.0;
  if (L.M > 0 && G) {
    const int box = (j / L.n) * L.nb + (i / L.n);
    const int* org = L.orgB + comp * L.M * 2;
    const double* wb = L.wB + (size_t)comp * L.M * IBMG_PATCH;
    for (int q = L.box_start[box]; q < L.box_start[box + 1]; ++q) {
      const int k = L.box_list[q];
      const int di = (i - org[2 * k]) & msk, dj = (j - org[2 * k + 1]) & msk;
      if (di < 4 && dj < 4) sp += wb[k * IBMG_PATCH + dj * 4 + di] * G[2 * k + comp];
    }
  }
  val += sp * inv_h2;
  if (g0) val += g0[rem];
  b[idx] = val;
}

// ---------------------------------------------------------------- a14: U = S^* u, X += dt U
__global__ void __launch_bounds__(256)
k_interp(LevelView<double> L, const double* __restrict__ u, const double* __restrict__ v,
         double* __restrict__ U, double* __restrict__ X, double dt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * L.M) return;
  const int comp = t / L.M, k = t - comp * L.M;
  const int N = L.N, msk = N - 1;
  const double* f = comp == 0 ? u : v;
  const int oi = L.orgC[2 * t], oj = L.orgC[2 * t + 1];
  const double* wc = L.wC + (size_t)t * IBMG_PATCH;
  double acc = 0.0;
  for (int e = 0; e < 16; ++e) acc += wc[e] * f[((oj + (e >> 2)) & msk) * N + ((oi + (e & 3)) & msk)];
  if (U) U[2 * k + comp] = acc;
  if (X) X[2 * k + comp] += dt * acc;
}

// ---------------------------------------------------------------- launchers
namespace ibmg {

template <typename T> void launch_gather(hipStream_t s, const LevelView<T>& L, const T* w) {
  if (L.M > 0) k_gather<T><<<nblk(2 * L.M), 256, 0, s>>>(L, w);
}
template <typename T> void launch_residual(hipStream_t s, const LevelView<T>& L, const T* b, const T* w, T* r,
                                           bool ib) {
  k_residual<T><<<nblk(3 * (size_t)L.N * L.N), 256, 0, s>>>(L, b, w, r, ib ? 1 : 0);
}
template <typename T> void launch_phase(hipStream_t s, const LevelView<T>& L, const T* b, T* w, int colour,
                                        bool ib) {
  LevelView<T> V = L;
  if (!ib) V.ib_index = nullptr;
  const int half = L.nb / 2;
  k_phase<T><<<half * half, 64, 0, s>>>(V, b, w, colour & 1, colour >> 1);
}
template <typename T> void launch_restrict(hipStream_t s, int Nf, const T* rf, T* rc) {
  k_restrict<T><<<nblk(3 * (size_t)(Nf / 2) * (Nf / 2)), 256, 0, s>>>(Nf, rf, rc);
}
template <typename T> void launch_prolong_add(hipStream_t s, int Nf, const T* ec, T* wf) {
  k_prolong_add<T><<<nblk(3 * (size_t)Nf * Nf), 256, 0, s>>>(Nf, ec, wf);
}
void launch_rhs(hipStream_t s, const LevelView<double>& L0, double inv_h2, const double* u, const double* v,
                const double* gu, const double* gv, const double* G, double* b) {
  k_rhs<<<nblk(3 * (size_t)L0.N * L0.N), 256, 0, s>>>(L0, inv_h2, u, v, gu, gv, G, b);
}
void launch_interp(hipStream_t s, const LevelView<double>& L0, const double* u, const double* v, double* U,
                   double* X, double dt) {
  if (L0.M > 0) k_interp<<<nblk(2 * L0.M), 256, 0, s>>>(L0, u, v, U, X, dt);
}

#define IBMG_INST(T)                                                                                    \
  template void launch_gather<T>(hipStream_t, const LevelView<T>&, const T*);                          \
  template void launch_residual<T>(hipStream_t, const LevelView<T>&, const T*, const T*, T*, bool);     \
  template void launch_phase<T>(hipStream_t, const LevelView<T>&, const T*, T*, int, bool);             \
  template void launch_restrict<T>(hipStream_t, int, const T*, T*);                                     \
  template void launch_prolong_add<T>(hipStream_t, int, const T*, T*);
IBMG_INST(double)
IBMG_INST(float)
#undef IBMG_INST

}  // namespace ibmg
