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

}  // namespace ibmg
