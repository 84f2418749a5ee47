// Learned initial iterate for the per-step FGMRES solve (Sec. 3.3 starts the
// Krylov iteration from an initial iterate; this network proposes it as
// x0 = w^n + Dw).  Six 3x3 periodic convolutions, channels
// 5 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3, ReLU between layers; inputs
// (u, v, p, f_u, f_v) / s_in as index-aligned planes, output Dw / s_out.
//
// gfx950 mapping:
//   - activations and gradient planes are BF16, pixel-major with the
//     channels contiguous (16 or 32 per pixel);
//   - forward and backward-data convolutions are implicit GEMMs on the
//     16x16x16 BF16 MFMA with FP32 accumulation: a wavefront owns 64
//     consecutive pixels (four M tiles) and every output channel (one or two
//     N tiles), the K loop runs over the 9 taps and 16-channel chunks;
//   - weight gradients are FP32 sums over pixel chunks (fixed partition,
//     fixed-order reduction, so training is deterministic);
//   - masters, Adam moments and the loss are FP32; every update rewrites
//     the BF16 forward weights and the flipped, transposed BF16 weights of
//     the backward-data pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ibmg.h"
#include "common.h"
#include "kernels.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

constexpr int kLayers = 6;
constexpr int kCin[kLayers] = {5, 32, 32, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 32, 32, 3};
constexpr int kCinP[kLayers] = {16, 32, 32, 32, 32, 32};    // padded to the MFMA K chunk
constexpr int kCoutP[kLayers] = {32, 32, 32, 32, 32, 16};   // padded to the MFMA N tile
constexpr int kPix = 1024;        // pixels per weight-gradient chunk
constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;

__host__ __device__ constexpr int layer_params(int l) { return kCout[l] * kCin[l] * 9 + kCout[l]; }
constexpr int param_offset(int l) { return l == 0 ? 0 : param_offset(l - 1) + layer_params(l - 1); }
constexpr int kParams = param_offset(kLayers);
static_assert(kParams == 39331, "5-32-32-32-32-32-3 network with 3x3 kernels");

__device__ inline bf16_t to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ inline float from_bf16(bf16_t h) { return __uint_as_float((unsigned)h << 16); }

// ---------------------------------------------------------------- convolution on MFMA
// out(p, o) = sum_{tap, c} W[tap][o][c] in(shift_tap(p), c), taps (ky, kx)
// read at (y + ky - 1, x + kx - 1), periodic.  CIP input channels per pixel,
// COP output channels.  MODE 0: + bias, ReLU, BF16 out [P][COP];
// MODE 1: + bias, FP32 planes out[o][p] for o < nout; MODE 2: times the mask
// (mask(p, o) > 0), BF16 out [P][COP] (backward data through a ReLU).
template <int CIP, int COP, int MODE>
__global__ void __launch_bounds__(256)
k_conv(int N, const bf16_t* __restrict__ in, const bf16_t* __restrict__ w, const float* __restrict__ bias,
       const bf16_t* __restrict__ mask, bf16_t* __restrict__ out_h, float* __restrict__ out_f, int nout) {
  constexpr int NT = COP / 16, KC = CIP / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int P = N * N, msk = N - 1, lg = __builtin_ctz(N);
  const int p0 = (blockIdx.x * 4 + wave) * 64;
  if (p0 >= P) return;
  const int row16 = lane & 15, kq = lane >> 4;   // A/B: row (or column) within a tile, K quarter
  v4f acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
  int py[4], px[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int p = p0 + mt * 16 + row16;
    py[mt] = p >> lg;
    px[mt] = p & msk;
  }
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    int q[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) q[mt] = ((py[mt] + dy) & msk) * N + ((px[mt] + dx) & msk);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int c0 = kc * 16 + kq * 4;
      v4s b[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = *reinterpret_cast<const v4s*>(w + ((size_t)tap * COP + nt * 16 + row16) * CIP + c0);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const v4s a = *reinterpret_cast<const v4s*>(in + (size_t)q[mt] * CIP + c0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nt], acc[mt][nt], 0, 0, 0);
      }
    }
  }
  // D(m, n): lane holds rows m = 4 * kq + i, column n = row16
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = p0 + mt * 16 + kq * 4 + i;
        const int o = nt * 16 + row16;
        float v = acc[mt][nt][i];
        if (MODE == 0) {
          v += bias[o];
          out_h[(size_t)p * COP + o] = to_bf16(v > 0.f ? v : 0.f);
        } else if (MODE == 1) {
          if (o < nout) out_f[(size_t)o * P + p] = v + bias[o];
        } else {
          out_h[(size_t)p * COP + o] = to_bf16(from_bf16(mask[(size_t)p * COP + o]) > 0.f ? v : 0.f);
        }
      }
}

// ---------------------------------------------------------------- weight gradients
// part[chunk][tap][o][c] = sum over the chunk's pixels p of g(p, o) a(shift_tap(p), c);
// partb[chunk][o] = sum of g(p, o) (tap-0 blocks).  g: [P][GP] BF16, a: [P][AP].
__global__ void __launch_bounds__(256)
k_wgrad(int N, const bf16_t* __restrict__ g, int GP, int co, const bf16_t* __restrict__ a, int AP, int ci,
        float* __restrict__ part, float* __restrict__ partb) {
  __shared__ float sg[16][32];
  __shared__ float sa[16][32];
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int P = N * N, msk = N - 1, lg = __builtin_ctz(N);
  const int t = threadIdx.x;
  // thread -> (o, c0..c0+3)
  const int o = t >> 3, c0 = (t & 7) * 4;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;
  const int pbeg = chunk * kPix, pend = min(P, pbeg + kPix);
  for (int pb = pbeg; pb < pend; pb += 16) {
    // stage 16 pixels of g and of the shifted a
    for (int e = t; e < 16 * 32; e += 256) {
      const int k = e >> 5, c = e & 31;
      const int p = pb + k;
      float gv = 0.f, av = 0.f;
      if (p < pend) {
        if (c < co) gv = from_bf16(g[(size_t)p * GP + c]);
        if (c < ci) {
          const int y = p >> lg, x = p & msk;
          const int q = ((y + dy) & msk) * N + ((x + dx) & msk);
          av = from_bf16(a[(size_t)q * AP + c]);
        }
      }
      sg[k][c] = gv;
      sa[k][c] = av;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float gv = sg[k][o];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += gv * sa[k][c0 + j];
      if (tap == 0 && (t & 7) == 0) accb += gv;
    }
    __syncthreads();
  }
  float* dst = part + (((size_t)chunk * 9 + tap) * 32 + o) * 32 + c0;
#pragma unroll
  for (int j = 0; j < 4; ++j) dst[j] = acc[j];
  if (tap == 0 && (t & 7) == 0) partb[(size_t)chunk * 32 + o] = accb;
}

// grad[poff + ...] = sum over chunks (ascending) of the partials, in the flat
// parameter packing (W [co][ci][ky][kx], then b [co]).
__global__ void __launch_bounds__(256)
k_wgrad_reduce(int nchunk, const float* __restrict__ part, const float* __restrict__ partb, int co, int ci,
               float* __restrict__ grad) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = co * ci * 9;
  if (idx >= nw + co) return;
  float s = 0.f;
  if (idx < nw) {
    const int o = idx / (ci * 9), rem = idx - o * ci * 9, c = rem / 9, tap = rem - c * 9;
    for (int k = 0; k < nchunk; ++k) s += part[(((size_t)k * 9 + tap) * 32 + o) * 32 + c];
  } else {
    const int o = idx - nw;
    for (int k = 0; k < nchunk; ++k) s += partb[(size_t)k * 32 + o];
  }
  grad[idx] = s;
}

// ---------------------------------------------------------------- packing, loss, Adam
// Network input: in5 (five FP64 planes) / s_in -> BF16 [P][16] (channels 5..15 zero).
__global__ void __launch_bounds__(256)
k_pack_in(int P, const double* __restrict__ in5, const float* __restrict__ s_in, bf16_t* __restrict__ a0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  for (int c = 0; c < 16; ++c)
    a0[(size_t)p * 16 + c] = c < 5 ? to_bf16((float)(in5[(size_t)c * P + p] / (double)s_in[c])) : (bf16_t)0;
}

// Same from a stored FP32 pair (planes [8][P]: five inputs, three targets).
__global__ void __launch_bounds__(256)
k_pack_pair(int P, const float* __restrict__ pair, const float* __restrict__ s_in, bf16_t* __restrict__ a0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  for (int c = 0; c < 16; ++c) a0[(size_t)p * 16 + c] = c < 5 ? to_bf16(pair[(size_t)c * P + p] / s_in[c]) : (bf16_t)0;
}

// dz6 = 2 (y - t / s_out) / (3 P) (BF16 [P][16]); partial[block] = sum of (y - t/s)^2.
__global__ void __launch_bounds__(256)
k_loss(int P, const float* __restrict__ y, const float* __restrict__ tgt, const float* __restrict__ s_out,
       bf16_t* __restrict__ dz, float* __restrict__ partial) {
  __shared__ float sh[256];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (p < P) {
    const float inv = 2.f / (3.f * (float)P);
    for (int c = 0; c < 16; ++c) {
      float gv = 0.f;
      if (c < 3) {
        const float d = y[(size_t)c * P + p] - tgt[(size_t)c * P + p] / s_out[c];
        l += d * d;
        gv = inv * d;
      }
      dz[(size_t)p * 16 + c] = to_bf16(gv);
    }
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// loss_acc[0] += (sum of partials) / (3 P)
__global__ void k_loss_sum(int nb, const float* __restrict__ partial, int P, float* __restrict__ loss_acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += partial[b];
  loss_acc[0] += s / (3.f * (float)P);
}

struct WeightViews {
  bf16_t* wf[kLayers];
  bf16_t* wb[kLayers];
  float* bias[kLayers];
};

// Write parameter idx of the flat vector into the BF16 forward/backward
// weights or the bias array.
__device__ inline void scatter_param(const WeightViews& V, int idx, float val) {
  int l = 0;
  while (l + 1 < kLayers && idx >= param_offset(l + 1)) ++l;
  const int r = idx - param_offset(l);
  const int nw = kCout[l] * kCin[l] * 9;
  if (r < nw) {
    const int o = r / (kCin[l] * 9), rem = r - o * kCin[l] * 9, c = rem / 9, tap = rem - c * 9;
    const bf16_t h = to_bf16(val);
    V.wf[l][((size_t)tap * kCoutP[l] + o) * kCinP[l] + c] = h;
    // backward data: tap' = 8 - tap (flip), roles of o and c exchanged
    V.wb[l][((size_t)(8 - tap) * kCinP[l] + c) * kCoutP[l] + o] = h;
  } else {
    V.bias[l][r - nw] = val;
  }
}

__global__ void __launch_bounds__(256) k_scatter(int n, const float* __restrict__ theta, WeightViews V) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) scatter_param(V, idx, theta[idx]);
}

__global__ void __launch_bounds__(256)
k_adam(int n, float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
       float lr, float c1, float c2, WeightViews V) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const float gi = g[idx];
  const float mi = kB1 * m[idx] + (1.f - kB1) * gi;
  const float vi = kB2 * v[idx] + (1.f - kB2) * gi * gi;
  m[idx] = mi;
  v[idx] = vi;
  const float t = theta[idx] - lr * (mi / c1) / (sqrtf(vi / c2) + kEps);
  theta[idx] = t;
  scatter_param(V, idx, t);
}

// Per-channel RMS over the recorded pairs: acc[c] = sum over pairs and pixels of x^2.
__global__ void __launch_bounds__(256)
k_sumsq(int P, int npairs, const float* __restrict__ pairs, double* __restrict__ acc) {
  __shared__ double sh[256];
  const int c = blockIdx.x;    // 0..7
  double s = 0.0;
  for (int k = 0; k < npairs; ++k)
    for (int p = threadIdx.x; p < P; p += 256) {
      const double x = pairs[((size_t)k * 8 + c) * P + p];
      s += x * x;
    }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[c] = sh[0];
}

__global__ void k_scales(const double* __restrict__ acc, double count, float* __restrict__ s) {
  const int c = threadIdx.x;
  if (c >= 8) return;
  const double r = sqrt(acc[c] / count);
  s[c] = r > 0.0 ? (float)r : 1.f;
}

__global__ void __launch_bounds__(256)
k_store_pair(int P, const double* __restrict__ in5, const double* __restrict__ dw3, float* __restrict__ pair) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 8 * P) return;
  const int c = idx / P, p = idx - c * P;
  pair[idx] = (float)(c < 5 ? in5[(size_t)c * P + p] : dw3[(size_t)(c - 5) * P + p]);
}

__global__ void __launch_bounds__(256)
k_unpack_out(int P, const float* __restrict__ y, const float* __restrict__ s_out, double* __restrict__ dw3) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * P) return;
  dw3[idx] = (double)y[idx] * (double)s_out[idx / P];
}

}  // namespace

// ====================================================================== handle
struct ibmg_cnn {
  int N = 0, P = 0, max_pairs = 0, npairs = 0, nchunk = 0;
  int64_t nrec = 0;   // pairs recorded so far (the store keeps the last max_pairs)
  int64_t adam_t = 0;
  bool scales_set = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t need = 0;
  size_t o_theta = 0, o_m = 0, o_v = 0, o_grad = 0, o_wf[kLayers] = {}, o_wb[kLayers] = {}, o_bias[kLayers] = {};
  size_t o_act[kLayers] = {}, o_dz[2] = {}, o_y = 0, o_part = 0, o_partb = 0, o_lpart = 0, o_loss = 0;
  size_t o_scale = 0, o_sumsq = 0, o_pairs = 0;
  size_t o_traj = 0;   // features (6 planes), w^n, dw^{n-1}, proposal, dw^n (3 planes each), FP64
  template <typename T> T* d(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  WeightViews views() const {
    WeightViews V;
    for (int l = 0; l < kLayers; ++l) {
      V.wf[l] = d<bf16_t>(o_wf[l]);
      V.wb[l] = d<bf16_t>(o_wb[l]);
      V.bias[l] = d<float>(o_bias[l]);
    }
    return V;
  }
};

namespace {

using namespace ibmg;

void forward(ibmg_cnn* C) {
  hipStream_t s = C->stream;
  const int N = C->N, P = C->P;
  const unsigned grid = (unsigned)((P + 255) / 256);
  const WeightViews V = C->views();
  k_conv<16, 32, 0><<<grid, 256, 0, s>>>(N, C->d<bf16_t>(C->o_act[0]), V.wf[0], V.bias[0], nullptr,
                                         C->d<bf16_t>(C->o_act[1]), nullptr, 0);
  for (int l = 1; l < kLayers - 1; ++l)
    k_conv<32, 32, 0><<<grid, 256, 0, s>>>(N, C->d<bf16_t>(C->o_act[l]), V.wf[l], V.bias[l], nullptr,
                                           C->d<bf16_t>(C->o_act[l + 1]), nullptr, 0);
  k_conv<32, 16, 1><<<grid, 256, 0, s>>>(N, C->d<bf16_t>(C->o_act[kLayers - 1]), V.wf[kLayers - 1],
                                         V.bias[kLayers - 1], nullptr, nullptr, C->d<float>(C->o_y), 3);
}

// Loss and gradient of the pair whose input is packed in act[0] and whose
// target planes are tgt; grad (flat) in o_grad, loss added to o_loss.
void backward(ibmg_cnn* C, const float* tgt) {
  hipStream_t s = C->stream;
  const int N = C->N, P = C->P;
  const unsigned grid = (unsigned)((P + 255) / 256);
  const WeightViews V = C->views();
  k_loss<<<grid, 256, 0, s>>>(P, C->d<float>(C->o_y), tgt, C->d<float>(C->o_scale) + 5, C->d<bf16_t>(C->o_dz[0]),
                               C->d<float>(C->o_lpart));
  k_loss_sum<<<1, 64, 0, s>>>((int)grid, C->d<float>(C->o_lpart), P, C->d<float>(C->o_loss));
  int cur = 0;   // dz[cur] holds dL/dz_l ([P][coutp])
  for (int l = kLayers - 1; l >= 0; --l) {
    const bf16_t* g = C->d<bf16_t>(C->o_dz[cur]);
    k_wgrad<<<dim3(C->nchunk, 9), 256, 0, s>>>(N, g, kCoutP[l], kCout[l], C->d<bf16_t>(C->o_act[l]), kCinP[l],
                                                kCin[l], C->d<float>(C->o_part), C->d<float>(C->o_partb));
    const int np = layer_params(l);
    k_wgrad_reduce<<<nblk(np), 256, 0, s>>>(C->nchunk, C->d<float>(C->o_part), C->d<float>(C->o_partb), kCout[l],
                                            kCin[l], C->d<float>(C->o_grad) + param_offset(l));
    if (l == 0) break;
    bf16_t* gn = C->d<bf16_t>(C->o_dz[1 - cur]);
    if (l == kLayers - 1)
      k_conv<16, 32, 2><<<grid, 256, 0, s>>>(N, g, V.wb[l], nullptr, C->d<bf16_t>(C->o_act[l]), gn, nullptr, 0);
    else
      k_conv<32, 32, 2><<<grid, 256, 0, s>>>(N, g, V.wb[l], nullptr, C->d<bf16_t>(C->o_act[l]), gn, nullptr, 0);
    cur = 1 - cur;
  }
}

int compute_scales(ibmg_cnn* C) {
  if (C->scales_set) return IBMG_OK;
  if (C->npairs == 0) return IBMG_ESTATE;
  hipStream_t s = C->stream;
  k_sumsq<<<8, 256, 0, s>>>(C->P, C->npairs, C->d<float>(C->o_pairs), C->d<double>(C->o_sumsq));
  k_scales<<<1, 64, 0, s>>>(C->d<double>(C->o_sumsq), (double)C->npairs * C->P, C->d<float>(C->o_scale));
  IBMG_HIP(hipGetLastError());
  C->scales_set = true;
  return IBMG_OK;
}

}  // namespace

namespace ibmg {

int cnn_traj(ibmg_cnn* C, CnnTraj* t) {
  if (!C || !C->ws || !t) return IBMG_ENOMEM;
  const size_t P = C->P;
  double* base = C->d<double>(C->o_traj);
  t->N = C->N;
  t->stream = C->stream;
  t->feat = base;
  t->wold = base + 6 * P;
  t->dprev = base + 9 * P;
  t->x0 = base + 12 * P;
  t->dw = base + 15 * P;
  return IBMG_OK;
}

}  // namespace ibmg

extern "C" {

int ibmg_guess_reset(ibmg_cnn* C) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  // a new trajectory: no previous increment
  k_fill<double><<<nblk(3 * (size_t)C->P), 256, 0, C->stream>>>(C->d<double>(C->o_traj) + 9 * (size_t)C->P,
                                                                 3 * (size_t)C->P, 0.0);
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

int ibmg_guess_get_increment(ibmg_cnn* C, double* dw3) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!dw3) return IBMG_EINVAL;
  IBMG_HIP(hipMemcpyAsync(dw3, C->d<double>(C->o_traj) + 9 * (size_t)C->P, 3 * (size_t)C->P * sizeof(double),
                          hipMemcpyDeviceToDevice, C->stream));
  IBMG_HIP(hipStreamSynchronize(C->stream));
  return IBMG_OK;
}

int ibmg_guess_set_increment(ibmg_cnn* C, const double* dw3) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!dw3) return IBMG_EINVAL;
  IBMG_HIP(hipMemcpyAsync(C->d<double>(C->o_traj) + 9 * (size_t)C->P, dw3, 3 * (size_t)C->P * sizeof(double),
                          hipMemcpyDeviceToDevice, C->stream));
  return IBMG_OK;
}

int ibmg_cnn_create(ibmg_cnn** out, int32_t N, int32_t max_pairs, void* stream) {
  if (!out) return IBMG_EINVAL;
  *out = nullptr;
  if (N < 16 || N > 4096 || (N & (N - 1))) return IBMG_ESHAPE;
  if (max_pairs < 1) return IBMG_EINVAL;
  ibmg_cnn* C = new (std::nothrow) ibmg_cnn();
  if (!C) return IBMG_EINVAL;
  C->N = N;
  C->P = N * N;
  C->max_pairs = max_pairs;
  C->nchunk = (C->P + kPix - 1) / kPix;
  C->stream = (hipStream_t)stream;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    cur = (cur + 255) & ~(size_t)255;
    const size_t o = cur;
    cur += bytes;
    return o;
  };
  const size_t P = C->P;
  C->o_theta = take(kParams * sizeof(float));
  C->o_m = take(kParams * sizeof(float));
  C->o_v = take(kParams * sizeof(float));
  C->o_grad = take(kParams * sizeof(float));
  for (int l = 0; l < kLayers; ++l) {
    C->o_wf[l] = take(9 * (size_t)kCoutP[l] * kCinP[l] * sizeof(bf16_t));
    C->o_wb[l] = take(9 * (size_t)kCoutP[l] * kCinP[l] * sizeof(bf16_t));
    C->o_bias[l] = take(kCoutP[l] * sizeof(float));
    C->o_act[l] = take(P * kCinP[l] * sizeof(bf16_t));
  }
  C->o_dz[0] = take(P * 32 * sizeof(bf16_t));
  C->o_dz[1] = take(P * 32 * sizeof(bf16_t));
  C->o_y = take(3 * P * sizeof(float));
  C->o_part = take((size_t)C->nchunk * 9 * 32 * 32 * sizeof(float));
  C->o_partb = take((size_t)C->nchunk * 32 * sizeof(float));
  C->o_lpart = take(((P + 255) / 256) * sizeof(float));
  C->o_loss = take(4 * sizeof(float));
  C->o_scale = take(8 * sizeof(float));
  C->o_sumsq = take(8 * sizeof(double));
  C->o_traj = take(18 * P * sizeof(double));   // zeroed at bind: dw^{-1} = 0
  C->o_pairs = take((size_t)max_pairs * 8 * P * sizeof(float));
  C->need = cur + 256;
  *out = C;
  return IBMG_OK;
}

int ibmg_cnn_workspace_bytes(const ibmg_cnn* C, size_t* bytes) {
  if (!C || !bytes) return IBMG_EINVAL;
  *bytes = C->need;
  return IBMG_OK;
}

int ibmg_cnn_bind_workspace(ibmg_cnn* C, void* dev, size_t bytes) {
  if (!C || !dev) return IBMG_EINVAL;
  char* base = (char*)(((uintptr_t)dev + 255) & ~(uintptr_t)255);
  if (bytes < C->need || (size_t)(base - (char*)dev) + C->need - 256 > bytes) return IBMG_ENOMEM;
  C->ws = base;
  // zero everything up to the pair store (padding of the BF16 weights stays zero)
  IBMG_HIP(hipMemsetAsync(C->ws, 0, C->o_pairs, C->stream));
  IBMG_HIP(hipStreamSynchronize(C->stream));
  C->npairs = 0;
  C->nrec = 0;
  C->adam_t = 0;
  C->scales_set = false;
  return IBMG_OK;
}

int ibmg_cnn_set_params(ibmg_cnn* C, const float* host) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!host) return IBMG_EINVAL;
  hipStream_t s = C->stream;
  IBMG_HIP(hipMemcpyAsync(C->d<float>(C->o_theta), host, kParams * sizeof(float), hipMemcpyHostToDevice, s));
  IBMG_HIP(hipMemsetAsync(C->d<float>(C->o_m), 0, kParams * sizeof(float), s));
  IBMG_HIP(hipMemsetAsync(C->d<float>(C->o_v), 0, kParams * sizeof(float), s));
  k_scatter<<<nblk(kParams), 256, 0, s>>>(kParams, C->d<float>(C->o_theta), C->views());
  IBMG_HIP(hipGetLastError());
  IBMG_HIP(hipStreamSynchronize(s));
  C->adam_t = 0;
  return IBMG_OK;
}

int ibmg_cnn_get_params(ibmg_cnn* C, float* host) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!host) return IBMG_EINVAL;
  IBMG_HIP(hipMemcpyAsync(host, C->d<float>(C->o_theta), kParams * sizeof(float), hipMemcpyDeviceToHost, C->stream));
  IBMG_HIP(hipStreamSynchronize(C->stream));
  return IBMG_OK;
}

int ibmg_cnn_set_scales(ibmg_cnn* C, const float* s_in5, const float* s_out3) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!s_in5 || !s_out3) return IBMG_EINVAL;
  float s[8];
  for (int c = 0; c < 5; ++c) s[c] = s_in5[c];
  for (int c = 0; c < 3; ++c) s[5 + c] = s_out3[c];
  for (float x : s)
    if (!(x > 0.f) || !std::isfinite(x)) return IBMG_EINVAL;
  IBMG_HIP(hipMemcpyAsync(C->d<float>(C->o_scale), s, sizeof(s), hipMemcpyHostToDevice, C->stream));
  IBMG_HIP(hipStreamSynchronize(C->stream));
  C->scales_set = true;
  return IBMG_OK;
}

int ibmg_cnn_get_scales(ibmg_cnn* C, float* s8) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!s8) return IBMG_EINVAL;
  IBMG_HIP(hipMemcpyAsync(s8, C->d<float>(C->o_scale), 8 * sizeof(float), hipMemcpyDeviceToHost, C->stream));
  IBMG_HIP(hipStreamSynchronize(C->stream));
  return IBMG_OK;
}

int ibmg_cnn_record(ibmg_cnn* C, const double* in5, const double* dw3) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!in5 || !dw3) return IBMG_EINVAL;
  const int slot = (int)(C->nrec % C->max_pairs);
  float* dst = C->d<float>(C->o_pairs) + (size_t)slot * 8 * C->P;
  k_store_pair<<<nblk(8 * (size_t)C->P), 256, 0, C->stream>>>(C->P, in5, dw3, dst);
  IBMG_HIP(hipGetLastError());
  ++C->nrec;
  C->npairs = (int)std::min<int64_t>(C->nrec, C->max_pairs);
  return IBMG_OK;
}

int ibmg_cnn_pairs(const ibmg_cnn* C, int32_t* n) {
  if (!C || !n) return IBMG_EINVAL;
  *n = C->npairs;
  return IBMG_OK;
}

int ibmg_cnn_train(ibmg_cnn* C, int32_t epochs, float lr, float* loss_first, float* loss_last) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (epochs < 1 || !(lr > 0.f)) return IBMG_EINVAL;
  if (C->npairs == 0) return IBMG_ESTATE;
  int rc = compute_scales(C);
  if (rc) return rc;
  hipStream_t s = C->stream;
  const unsigned grid = (unsigned)((C->P + 255) / 256);
  float lf = 0.f, ll = 0.f;
  for (int e = 0; e < epochs; ++e) {
    IBMG_HIP(hipMemsetAsync(C->d<float>(C->o_loss), 0, sizeof(float), s));
    for (int k = 0; k < C->npairs; ++k) {
      const float* pair = C->d<float>(C->o_pairs) + (size_t)k * 8 * C->P;
      k_pack_pair<<<grid, 256, 0, s>>>(C->P, pair, C->d<float>(C->o_scale), C->d<bf16_t>(C->o_act[0]));
      forward(C);
      backward(C, pair + (size_t)5 * C->P);
      ++C->adam_t;
      const float c1 = 1.f - std::pow(kB1, (float)C->adam_t), c2 = 1.f - std::pow(kB2, (float)C->adam_t);
      k_adam<<<nblk(kParams), 256, 0, s>>>(kParams, C->d<float>(C->o_theta), C->d<float>(C->o_m),
                                           C->d<float>(C->o_v), C->d<float>(C->o_grad), lr, c1, c2, C->views());
    }
    float lsum = 0.f;
    IBMG_HIP(hipMemcpyAsync(&lsum, C->d<float>(C->o_loss), sizeof(float), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    if (e == 0) lf = lsum / C->npairs;
    ll = lsum / C->npairs;
  }
  IBMG_HIP(hipGetLastError());
  if (loss_first) *loss_first = lf;
  if (loss_last) *loss_last = ll;
  return IBMG_OK;
}

int ibmg_cnn_infer(ibmg_cnn* C, const double* in5, double* dw3) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!in5 || !dw3) return IBMG_EINVAL;
  if (!C->scales_set) return IBMG_ESTATE;
  hipStream_t s = C->stream;
  k_pack_in<<<nblk(C->P), 256, 0, s>>>(C->P, in5, C->d<float>(C->o_scale), C->d<bf16_t>(C->o_act[0]));
  forward(C);
  k_unpack_out<<<nblk(3 * (size_t)C->P), 256, 0, s>>>(C->P, C->d<float>(C->o_y), C->d<float>(C->o_scale) + 5, dw3);
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

int ibmg_cnn_loss_grad(ibmg_cnn* C, const double* in5, const double* dw3, float* loss, float* grad_host) {
  if (!C || !C->ws) return IBMG_ENOMEM;
  if (!in5 || !dw3) return IBMG_EINVAL;
  if (!C->scales_set) return IBMG_ESTATE;
  hipStream_t s = C->stream;
  // the pair is staged as FP32 planes in the weight-gradient partial buffer
  // (9 P floats >= 8 P), packed, and its target planes moved to the second
  // gradient buffer before the backward pass reuses the partials
  float* tmp = C->d<float>(C->o_part);
  k_store_pair<<<nblk(8 * (size_t)C->P), 256, 0, s>>>(C->P, in5, dw3, tmp);
  k_pack_pair<<<nblk(C->P), 256, 0, s>>>(C->P, tmp, C->d<float>(C->o_scale), C->d<bf16_t>(C->o_act[0]));
  IBMG_HIP(hipMemsetAsync(C->d<float>(C->o_loss), 0, sizeof(float), s));
  forward(C);
  // dz[1] (32 P BF16 = 16 P floats) holds the 3 P target values until the
  // loss kernel has read them; the first backward convolution overwrites it
  float* t3 = reinterpret_cast<float*>(C->d<bf16_t>(C->o_dz[1]));
  IBMG_HIP(hipMemcpyAsync(t3, tmp + (size_t)5 * C->P, 3 * (size_t)C->P * sizeof(float), hipMemcpyDeviceToDevice,
                          s));
  backward(C, t3);
  IBMG_HIP(hipGetLastError());
  if (loss) IBMG_HIP(hipMemcpyAsync(loss, C->d<float>(C->o_loss), sizeof(float), hipMemcpyDeviceToHost, s));
  if (grad_host)
    IBMG_HIP(hipMemcpyAsync(grad_host, C->d<float>(C->o_grad), kParams * sizeof(float), hipMemcpyDeviceToHost, s));
  IBMG_HIP(hipStreamSynchronize(s));
  return IBMG_OK;
}

int ibmg_cnn_destroy(ibmg_cnn* C) {
  if (!C) return IBMG_EINVAL;
  delete C;
  return IBMG_OK;
}

}  // extern "C"
