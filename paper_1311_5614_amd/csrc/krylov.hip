// FGMRES building blocks on gfx950 (Sec. 3.3: multigrid as a right
// preconditioner for GMRES; the flexible form stores the preconditioned
// vectors).  All reductions are deterministic: a fixed grid-stride partition,
// a fixed LDS tree per workgroup, then a fixed tree over the partials.
#include "common.h"
#include "kernels.h"

#define MD_GROUP 8   // dot products per pass

// partial[(v) * nblocks + block] = block's share of <V[v], w>, v < nvec.
__global__ void __launch_bounds__(256)
k_multidot(const double* __restrict__ V, size_t ldv, int nvec, const double* __restrict__ w, size_t n,
           double* __restrict__ partial) {
  __shared__ double sh[MD_GROUP][256];
  const int g0 = blockIdx.y * MD_GROUP;
  const int ng = min(MD_GROUP, nvec - g0);
  double acc[MD_GROUP];
  // rows past the group's last vector repeat that vector: every load is
  // unconditional, so all of them are in flight together (their sums are
  // never stored)
  const double* Vq[MD_GROUP];
#pragma unroll
  for (int q = 0; q < MD_GROUP; ++q) {
    acc[q] = 0.0;
    Vq[q] = V + (size_t)(g0 + min(q, ng - 1)) * ldv;
  }
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const double we = w[e];
#pragma unroll
    for (int q = 0; q < MD_GROUP; ++q) acc[q] += Vq[q][e] * we;
  }
#pragma unroll
  for (int q = 0; q < MD_GROUP; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int q = 0; q < MD_GROUP; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + off];
    __syncthreads();
  }
  if ((int)threadIdx.x < ng) partial[(size_t)(g0 + threadIdx.x) * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

// out[v] (+)= sum of the nblocks partials of dot v (fixed tree).
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ partial, int nblocks, double* __restrict__ out, int accumulate) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) a += partial[(size_t)v * nblocks + b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = accumulate ? out[v] + sh[0] : sh[0];
}

// w[e] += sign * sum_v coef[v] V[v][e], v in fixed order.
__global__ void __launch_bounds__(256)
k_update(const double* __restrict__ V, size_t ldv, int nvec, const double* __restrict__ coef,
         double* __restrict__ w, size_t n, double sign) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  // unrolled so that eight basis loads are in flight; the sum keeps its order
#pragma unroll 8
  for (int v = 0; v < nvec; ++v) s += coef[v] * V[(size_t)v * ldv + e];
  w[e] += sign * s;
}

// out = w / sqrt(norm2[0]).
__global__ void __launch_bounds__(256)
k_scale(const double* __restrict__ w, double* __restrict__ out, size_t n, const double* __restrict__ norm2) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double nrm = sqrt(norm2[0]);
  out[e] = nrm > 0.0 ? w[e] / nrm : 0.0;
}

// Hessenberg storage is column-major: element (i, j) at H[j * ldh + i], so the
// dot products of column j land contiguously.  On entry H(j+1, j) holds the
// squared norm of the orthogonalised vector.  Applies the previous rotations
// to column j, forms the new one and updates g.  flags[0] = |g_{j+1}|,
// flags[1] = 1 if |g_{j+1}| <= target or the Arnoldi vector vanished,
// flags[2] = 1 on a non-finite value.
__global__ void k_givens(double* __restrict__ H, int ldh, double* __restrict__ g, double* __restrict__ cs,
                         double* __restrict__ sn, int j, double* __restrict__ flags, double target) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (size_t)j * ldh;
  const double hn = sqrt(col[j + 1]);
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double d = hypot(a, b);
  cs[j] = a / d;
  sn[j] = b / d;
  col[j] = d;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  const double est = fabs(g[j + 1]);
  flags[0] = est;
  flags[1] = (est <= target || hn == 0.0) ? 1.0 : 0.0;
  flags[2] = (isfinite(est) && isfinite(d)) ? 0.0 : 1.0;
}

// y = R^{-1} g over the leading k x k upper-triangular block.
__global__ void k_backsolve(const double* __restrict__ H, int ldh, const double* __restrict__ g, int k,
                            double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= H[(size_t)c * ldh + i] * y[c];
    y[i] = s / H[(size_t)i * ldh + i];
  }
}

// p -= sum / n (zero-mean pressure).
__global__ void __launch_bounds__(256) k_mean_shift(double* __restrict__ p, size_t n, const double* __restrict__ sum) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] -= sum[0] / (double)n;
}

// partial[b] = block b's share of sum(x).
__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ x, size_t n, double* __restrict__ partial) {
  __shared__ double sh[256];
  double a = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) a += x[e];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// out[0] = sum of the partials of one dot (fixed tree), also copied to copy[0].
__global__ void __launch_bounds__(256)
k_reduce2(const double* __restrict__ partial, int nblocks, double* __restrict__ out, double* __restrict__ copy) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) a += partial[b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = sh[0]; copy[0] = sh[0]; }
}

// w -= sum_v coef[v] V[v]; workgroup 0 also adds coef into acc (the second
// Gram-Schmidt pass's coefficients into the Hessenberg column).
__global__ void __launch_bounds__(256)
k_update_acc(const double* __restrict__ V, size_t ldv, int nvec, const double* __restrict__ coef,
             double* __restrict__ w, size_t n, double* __restrict__ acc) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (acc && blockIdx.x == 0)
    for (int t = threadIdx.x; t < nvec; t += blockDim.x) acc[t] += coef[t];
  if (e >= n) return;
  double s = 0.0;
  // unrolled so that eight basis loads are in flight; the sum keeps its order
#pragma unroll 8
  for (int v = 0; v < nvec; ++v) s += coef[v] * V[(size_t)v * ldv + e];
  w[e] -= s;
}

// v_{j+1} = w / sqrt(nrm2); workgroup 0 also performs the Givens step of
// column j (k_givens) -- the column's H(j+1, j) holds the same squared norm as
// nrm2, which every workgroup reads from nrm2.  The column and the previous
// rotations are first staged in LDS by the whole workgroup, so the serial
// chain of rotations (thread 0, same operations in the same order as
// k_givens) reads LDS instead of waiting on a global load per rotation.
constexpr int kGivensMax = 1024;  // >= the largest Krylov dimension + 2
__global__ void __launch_bounds__(256)
k_scale_givens(double* __restrict__ w, size_t n, const double* __restrict__ nrm2, double* __restrict__ H, int ldh,
               double* __restrict__ g, double* __restrict__ cs, double* __restrict__ sn, int j,
               double* __restrict__ flags, double target) {
  __shared__ double scol[kGivensMax], scs[kGivensMax], ssn[kGivensMax];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const double nrm = sqrt(nrm2[0]);
  if (e < n) w[e] = nrm > 0.0 ? w[e] / nrm : 0.0;
  if (blockIdx.x != 0) return;
  double* col = H + (size_t)j * ldh;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) scol[i] = col[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    scs[i] = cs[i];
    ssn[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    scol[j + 1] = nrm;
    for (int i = 0; i < j; ++i) {
      const double a = scol[i], b = scol[i + 1];
      scol[i] = scs[i] * a + ssn[i] * b;
      scol[i + 1] = -ssn[i] * a + scs[i] * b;
    }
    const double a = scol[j], b = scol[j + 1];
    const double d = hypot(a, b);
    cs[j] = a / d;
    sn[j] = b / d;
    scol[j] = d;
    scol[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double est = fabs(g[j + 1]);
    flags[0] = est;
    flags[1] = (est <= target || nrm == 0.0) ? 1.0 : 0.0;
    flags[2] = (isfinite(est) && isfinite(d)) ? 0.0 : 1.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) col[i] = scol[i];
}

// ---------------------------------------------------------------- delayed CGS2
// Classical Gram-Schmidt twice with the second projection delayed by one
// iteration: per iteration one pass over the basis forms the products of
// v_0 .. v_{j-1} and u_j (the previous iteration's once-projected, normalised
// vector) with u_j and with w = A z_j, and one pass completes u_j into v_j
// and projects w once against v_0 .. v_j.

// Sum over the 64 lanes of a wavefront (fixed butterfly: every lane ends with
// the same value, summed in the same order).
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

#define MD2_GROUP 16   // basis vectors per workgroup row of the two-vector product pass

// partial[v * nblocks + block] = block's share of <V[v], r1> (v < nvec) and
// partial[(nvec + v) * nblocks + block] of <V[v], r2>.
__global__ void __launch_bounds__(256)
k_multidot2(const double* __restrict__ V, size_t ldv, int nvec, const double* __restrict__ r1,
            const double* __restrict__ r2, size_t n, double* __restrict__ partial) {
  __shared__ double sh[2 * MD2_GROUP][4];
  const int g0 = blockIdx.y * MD2_GROUP;
  const int ng = min(MD2_GROUP, nvec - g0);
  double a1[MD2_GROUP], a2[MD2_GROUP];
  const double* Vq[MD2_GROUP];
#pragma unroll
  for (int q = 0; q < MD2_GROUP; ++q) {
    a1[q] = 0.0;
    a2[q] = 0.0;
    Vq[q] = V + (size_t)(g0 + min(q, ng - 1)) * ldv;   // past the group's end: its last vector again
  }
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const double x1 = r1[e], x2 = r2[e];
#pragma unroll
    for (int q = 0; q < MD2_GROUP; ++q) {
      const double vq = Vq[q][e];
      a1[q] += vq * x1;
      a2[q] += vq * x2;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < MD2_GROUP; ++q) {
    const double s1 = wave_sum(a1[q]), s2 = wave_sum(a2[q]);
    if (lane == 0) {
      sh[q][wave] = s1;
      sh[MD2_GROUP + q][wave] = s2;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * MD2_GROUP) {
    const int q = t % MD2_GROUP;
    if (q < ng) {
      const double v = (sh[t][0] + sh[t][1]) + (sh[t][2] + sh[t][3]);
      const size_t row = (t < MD2_GROUP) ? (size_t)(g0 + q) : (size_t)(nvec + g0 + q);
      partial[row * gridDim.x + blockIdx.x] = v;
    }
  }
}

// Sum over a 256-lane workgroup in a fixed order (wavefront butterflies, then
// the four wavefront sums in pairs); every thread returns the total.
__device__ inline double block_sum(double x, double* sh4) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = x;
  __syncthreads();
  const double tot = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return tot;
}

// Rotations 0 .. c-1 applied to column c (held in LDS as scol[0 .. c+1]),
// rotation c formed and g updated; thread 0 only, the operations and their
// order those of k_givens.
__device__ inline void rotate_column(double* scol, const double* scs, const double* ssn, int c, double* cs,
                                     double* sn, double* g) {
  for (int i = 0; i < c; ++i) {
    const double a = scol[i], b = scol[i + 1];
    scol[i] = scs[i] * a + ssn[i] * b;
    scol[i + 1] = -ssn[i] * a + scs[i] * b;
  }
  const double a = scol[c], b = scol[c + 1];
  const double d = hypot(a, b);
  cs[c] = a / d;
  sn[c] = b / d;
  scol[c] = d;
  scol[c + 1] = 0.0;
  g[c + 1] = -sn[c] * g[c];
  g[c] = cs[c] * g[c];
}

// One workgroup.  Completion of column jf >= 0: a[k] = <v_k, u_{jf+1}> for
// k <= jf and a[jf+1] = <u_{jf+1}, u_{jf+1}>; with t = a[0 .. jf] and
// rho = sqrt(a[jf+1] - |t|^2), u_{jf+1} = rho v_{jf+1} + sum_k t_k v_k, so
// column jf, which holds the first-pass products and H(jf+1, jf) = nu (the
// first-pass norm), gains nu t_k and H(jf+1, jf) = nu rho; its rotations are
// then applied and rotation jf formed.  Iteration mode (c given, j = jf + 1):
// c[k] = <v_k, w> for k < j and c[j] = <u_j, w>; column j receives the
// first-pass products H(k, j) = c[k] (k < j) and H(j, j) = s_j = <v_j, w> =
// (c[j] - t . c[0 .. j-1]) / rho, and coef = {1 / rho, s_j} for the update
// pass (jf = -1, j = 0: rho = 1, s_0 = c[0]).
__global__ void __launch_bounds__(256)
k_dcgs2_coef(const double* __restrict__ a, const double* __restrict__ c, int jf, double* __restrict__ H, int ldh,
             double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g, double* __restrict__ coef) {
  __shared__ double scol[kGivensMax], scs[kGivensMax], ssn[kGivensMax];
  __shared__ double sh4[4];
  double rho = 1.0, ts = 0.0;
  if (jf >= 0) {
    double p = 0.0, q = 0.0;
    for (int k = threadIdx.x; k <= jf; k += blockDim.x) {
      p += a[k] * a[k];
      if (c) q += a[k] * c[k];
    }
    const double tt = block_sum(p, sh4);
    ts = block_sum(q, sh4);
    rho = sqrt(a[jf + 1] - tt);
    double* col = H + (size_t)jf * ldh;
    const double nu = col[jf + 1];
    for (int k = threadIdx.x; k <= jf; k += blockDim.x) scol[k] = col[k] + nu * a[k];
    for (int k = threadIdx.x; k < jf; k += blockDim.x) {
      scs[k] = cs[k];
      ssn[k] = sn[k];
    }
    if (threadIdx.x == 0) scol[jf + 1] = nu * rho;
    __syncthreads();
    if (threadIdx.x == 0) rotate_column(scol, scs, ssn, jf, cs, sn, g);
    __syncthreads();
    for (int k = threadIdx.x; k <= jf + 1; k += blockDim.x) col[k] = scol[k];
  }
  if (!c) return;
  const int j = jf + 1;
  double* colj = H + (size_t)j * ldh;
  for (int k = threadIdx.x; k < j; k += blockDim.x) colj[k] = c[k];
  if (threadIdx.x == 0) {
    const double sj = rho > 0.0 ? (c[j] - ts) / rho : 0.0;
    colj[j] = sj;
    coef[0] = rho > 0.0 ? 1.0 / rho : 0.0;
    coef[1] = sj;
  }
}

// Per row e: v_j = (u_j - sum_{k<j} t_k v_k) / rho written over u_j, and
// w' = w - sum_{k<j} s_k v_k - s_j v_j written over w (coef = {1/rho, s_j});
// both sums share each basis load.  partial[block] = the block's share of
// |w'|^2.
__global__ void __launch_bounds__(256)
k_dcgs2_update(double* __restrict__ V, size_t ldv, int j, const double* __restrict__ t,
               const double* __restrict__ sc, const double* __restrict__ coef, size_t n,
               double* __restrict__ partial) {
  __shared__ double sh4[4];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (e < n) {
    double at = 0.0, as = 0.0;
    // unrolled so that eight basis loads are in flight; the sums keep their order
#pragma unroll 8
    for (int k = 0; k < j; ++k) {
      const double vk = V[(size_t)k * ldv + e];
      at += t[k] * vk;
      as += sc[k] * vk;
    }
    const double vj = (V[(size_t)j * ldv + e] - at) * coef[0];
    const double wp = V[(size_t)(j + 1) * ldv + e] - as - coef[1] * vj;
    V[(size_t)j * ldv + e] = vj;
    V[(size_t)(j + 1) * ldv + e] = wp;
    sq = wp * wp;
  }
  const double tot = block_sum(sq, sh4);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// u_{j+1} = w' / nu (nu = sqrt(nrm2[0])); workgroup 0 also writes H(j+1, j) =
// nu and the stopping test of column j on a rotated copy (rotations 0 .. j-1
// and the rotation column j would form): flags[0] = the residual estimate,
// flags[1] = 1 if it is <= target or nu = 0, flags[2] = 1 on a non-finite
// value.  H, the rotations and g are not changed.
__global__ void __launch_bounds__(256)
k_scale_tentative(double* __restrict__ w, size_t n, const double* __restrict__ nrm2, double* __restrict__ H,
                  int ldh, const double* __restrict__ g, const double* __restrict__ cs,
                  const double* __restrict__ sn, int j, double* __restrict__ flags, double target) {
  __shared__ double scol[kGivensMax], scs[kGivensMax], ssn[kGivensMax];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const double nrm = sqrt(nrm2[0]);
  if (e < n) w[e] = nrm > 0.0 ? w[e] / nrm : 0.0;
  if (blockIdx.x != 0) return;
  double* col = H + (size_t)j * ldh;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) scol[i] = col[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    scs[i] = cs[i];
    ssn[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    col[j + 1] = nrm;
    scol[j + 1] = nrm;
    for (int i = 0; i < j; ++i) {
      const double a = scol[i], b = scol[i + 1];
      scol[i] = scs[i] * a + ssn[i] * b;
      scol[i + 1] = -ssn[i] * a + scs[i] * b;
    }
    const double d = hypot(scol[j], scol[j + 1]);
    const double est = fabs(scol[j + 1] / d * g[j]);
    flags[0] = est;
    flags[1] = (est <= target || nrm == 0.0) ? 1.0 : 0.0;
    flags[2] = (isfinite(est) && isfinite(d)) ? 0.0 : 1.0;
  }
}

namespace ibmg {

void launch_multidot(hipStream_t s, const double* V, size_t ldv, int nvec, const double* w, size_t n,
                     double* partial, int nblocks) {
  dim3 grid(nblocks, (nvec + MD_GROUP - 1) / MD_GROUP);
  k_multidot<<<grid, 256, 0, s>>>(V, ldv, nvec, w, n, partial);
}
void launch_reduce(hipStream_t s, const double* partial, int nblocks, int nvec, double* out, int accumulate) {
  k_reduce<<<nvec, 256, 0, s>>>(partial, nblocks, out, accumulate);
}
void launch_update(hipStream_t s, const double* V, size_t ldv, int nvec, const double* coef, double* w,
                   size_t n, double sign) {
  k_update<<<nblk(n), 256, 0, s>>>(V, ldv, nvec, coef, w, n, sign);
}
void launch_scale(hipStream_t s, const double* w, double* out, size_t n, const double* norm2) {
  k_scale<<<nblk(n), 256, 0, s>>>(w, out, n, norm2);
}
void launch_givens(hipStream_t s, double* H, int ldh, double* g, double* cs, double* sn, int j, double* flags,
                   double target) {
  k_givens<<<1, 64, 0, s>>>(H, ldh, g, cs, sn, j, flags, target);
}
void launch_backsolve(hipStream_t s, const double* H, int ldh, const double* g, int k, double* y) {
  k_backsolve<<<1, 64, 0, s>>>(H, ldh, g, k, y);
}
void launch_mean_shift(hipStream_t s, double* p, size_t n, const double* sum) {
  k_mean_shift<<<nblk(n), 256, 0, s>>>(p, n, sum);
}
void launch_sum(hipStream_t s, const double* x, size_t n, double* partial, int nblocks) {
  k_sum<<<nblocks, 256, 0, s>>>(x, n, partial);
}
void launch_reduce2(hipStream_t s, const double* partial, int nblocks, double* out, double* copy) {
  k_reduce2<<<1, 256, 0, s>>>(partial, nblocks, out, copy);
}
void launch_update_acc(hipStream_t s, const double* V, size_t ldv, int nvec, const double* coef, double* w, size_t n,
                       double* acc) {
  k_update_acc<<<nblk(n), 256, 0, s>>>(V, ldv, nvec, coef, w, n, acc);
}
void launch_scale_givens(hipStream_t s, double* w, size_t n, const double* nrm2, double* H, int ldh, double* g,
                         double* cs, double* sn, int j, double* flags, double target) {
  k_scale_givens<<<nblk(n), 256, 0, s>>>(w, n, nrm2, H, ldh, g, cs, sn, j, flags, target);
}
void launch_multidot2(hipStream_t s, const double* V, size_t ldv, int nvec, const double* r1, const double* r2,
                      size_t n, double* partial, int nblocks) {
  dim3 grid(nblocks, (nvec + MD2_GROUP - 1) / MD2_GROUP);
  k_multidot2<<<grid, 256, 0, s>>>(V, ldv, nvec, r1, r2, n, partial);
}
void launch_dcgs2_coef(hipStream_t s, const double* a, const double* c, int jf, double* H, int ldh, double* cs,
                       double* sn, double* g, double* coef) {
  k_dcgs2_coef<<<1, 256, 0, s>>>(a, c, jf, H, ldh, cs, sn, g, coef);
}
void launch_dcgs2_update(hipStream_t s, double* V, size_t ldv, int j, const double* t, const double* sc,
                         const double* coef, size_t n, double* partial) {
  k_dcgs2_update<<<nblk(n), 256, 0, s>>>(V, ldv, j, t, sc, coef, n, partial);
}
void launch_scale_tentative(hipStream_t s, double* w, size_t n, const double* nrm2, double* H, int ldh,
                            const double* g, const double* cs, const double* sn, int j, double* flags,
                            double target) {
  k_scale_tentative<<<nblk(n), 256, 0, s>>>(w, n, nrm2, H, ldh, g, cs, sn, j, flags, target);
}

}  // namespace ibmg
