// Three-dimensional form of the method on gfx950 (include/ibmg3.h).
//
// Layout in HBM (per level l, N = N_l): a level vector is [u; v; w; p], each
// block N^3 doubles with flat index (k N + j) N + i.  The structure enters
// through per-point separable delta windows: S_l and J_l (the level's
// spreading and interpolation, S_0 = delta / h^3, J_0 = delta, S_{l+1} =
// R S_l, J_{l+1} = J_l P) are tensor products of one-dimensional transfers,
// so each (point, component) window is a base index and three 5-entry
// weight rows, kept in unwrapped coordinates and wrapped on use.  The
// elastic rows M_l x = S_l (-dt K L (J_l x)) are three passes: a gather per
// (point, component), the fibre second difference, and a gather per active
// face over the face's entries of a CSR of S_l, built once per setup from
// the points binned by window base (every sum has a fixed order).
//
// Box smoother: a box of n^3 cells has 3 (n + 1) n^2 + n^3 unknowns (304
// for n = 4).  The block of a box that meets no structure is the same for
// every box on a level (periodic, translation invariant), so its inverse is
// formed once per level and shared; each box that meets the structure gets
// its own dense inverse (assembled transposed, so that the in-place
// Gauss-Jordan inverse is the inverse stored column-major and the per-box
// product reads it with consecutive threads on consecutive rows).  A colour
// phase is a residual pass over the level (Jacobi within the colour) and
// one box pass.  FGMRES uses the delayed Gram-Schmidt kernels of krylov.hip.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ibmg3.h"
#include "common.h"
#include "handle.h"
#include "kernels.h"

namespace {

using ibmg::nblk;

constexpr int kW = 5;                 // window entries per axis on every level
constexpr int kBoxThreads = 512;      // box products: eight waves split the columns
constexpr int kGjThreads = 1024;      // box inverses
constexpr int kMaxNd = 3 * 5 * 16 + 64;   // 304: unknowns of an n = 4 box

struct Win {
  int base[3];
  double w[3][kW];
};

struct Lv3 {
  int N, n, nb, nd;
  double c, muh2, invh, coef, omega;   // coef = -dt K (0: no elastic rows)
  int M;
  const Win* S;            // [M * 3]
  const Win* J;            // [M * 3]
  const int* prev;
  const int* next;
  double* U;               // [M * 3]
  double* F;               // [M * 3]
  const int* bin_start;    // [3 N^3 + 1] points by wrapped S-window base, per component
  const int* bin_pts;      // [3 M]
  const int* act;          // [3 N^3] active faces (component * N^3 + face), ascending
  const int* nact;         // [1]
  const int* act_index;    // [3 N^3] index of a face in act, or -1
  const int* coff;         // [3 N^3 + 1] CSR of S_l by active face: offsets
  const int* cpt;          // point of each entry (ascending within a face)
  const double* cw;        // weight S_l(face, point) of each entry
  double* y;               // [3 N^3] elastic rows, zero off the active faces
};

__host__ __device__ inline int pmod(int a, int N) { return ((a % N) + N) % N; }
__host__ __device__ inline int floor_div2(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

// Sum of a window row's weights at grid index `coord` (all entries e with
// base + e = coord mod N; more than one only when N < kW).
__device__ inline double wsum(const Win& w, int d, int coord, int N) {
  double s = 0.0;
  for (int e = pmod(coord - w.base[d], N); e < kW; e += N) s += w.w[d][e];
  return s;
}

__device__ inline double wval(const Win& w, int i, int j, int k, int N) {
  const double a = wsum(w, 0, i, N);
  if (a == 0.0) return 0.0;
  const double b = wsum(w, 1, j, N);
  if (b == 0.0) return 0.0;
  return a * b * wsum(w, 2, k, N);
}

// Global index of local unknown t of box (bx, by, bz): families u, v, w with
// (n + 1) along their normal and n across, then the n^3 pressures; x fastest.
__device__ inline int box_dof(int t, int bx, int by, int bz, int n, int N) {
  const int nf = (n + 1) * n * n;
  const int fam = t < 3 * nf ? t / nf : 3;
  int r = fam < 3 ? t - fam * nf : t - 3 * nf;
  const int ex = fam == 0 ? n + 1 : n, ey = fam == 1 ? n + 1 : n;
  const int i = r % ex;
  r /= ex;
  const int j = r % ey, k = r / ey;
  const int gi = pmod(bx * n + i, N), gj = pmod(by * n + j, N), gk = pmod(bz * n + k, N);
  return fam * N * N * N + (gk * N + gj) * N + gi;
}

// Entry (row, col) of the re-discretised Stokes part of a level matrix
// (global unknown indices; periodic; neighbours counted with multiplicity).
__device__ double stokes_entry(const Lv3& L, int row, int col) {
  const int N = L.N, N3 = N * N * N;
  const int fr = row / N3, gr = row - fr * N3, fc = col / N3, gc = col - fc * N3;
  const int ri = gr % N, rj = (gr / N) % N, rk = gr / (N * N);
  auto shift = [&](int a, int s) {
    int i = ri, j = rj, k = rk;
    if (a == 0) i = pmod(i + s, N);
    else if (a == 1) j = pmod(j + s, N);
    else k = pmod(k + s, N);
    return (k * N + j) * N + i;
  };
  if (fr < 3) {
    if (fc == fr) {
      double v = gc == gr ? L.c + 6.0 * L.muh2 : 0.0;
      for (int a = 0; a < 3; ++a) {
        if (shift(a, 1) == gc) v -= L.muh2;
        if (shift(a, -1) == gc) v -= L.muh2;
      }
      return v;
    }
    if (fc == 3) return (gc == gr ? L.invh : 0.0) - (shift(fr, -1) == gc ? L.invh : 0.0);
    return 0.0;
  }
  if (fc < 3) return (gc == gr ? L.invh : 0.0) - (shift(fc, 1) == gc ? L.invh : 0.0);
  return 0.0;
}

// ---------------------------------------------------------------- windows

__global__ void __launch_bounds__(256) k3_win0(int M, int N, int kind, const double* __restrict__ X,
                                               Win* __restrict__ S, Win* __restrict__ J) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * M) return;
  const int p = t / 3, c = t - 3 * p;
  Win s, jw;
  for (int d = 0; d < 3; ++d) {
    const double off = d == c ? 0.0 : 0.5;
    const double x = X[3 * p + d] * N - off;
    const int b = (int)floor(x) - 1;
    s.base[d] = jw.base[d] = b;
    for (int e = 0; e < kW; ++e) {
      const double ph = e < 4 ? phi_kernel(x - (double)(b + e), kind) : 0.0;
      s.w[d][e] = ph * N;   // 1/h per axis: delta = phi phi phi / h^3
      jw.w[d][e] = ph;
    }
  }
  S[t] = s;
  J[t] = jw;
}

// One coarsening step of the windows, axis by axis: S_c = R S_f and
// J_c = J_f P with the one-dimensional factors of the face transfers
// (normal: restriction (1/4, 1/2, 1/4), linear prolongation; across:
// two-point average, 3/4-1/4 prolongation).
__global__ void __launch_bounds__(256) k3_win_coarse(int M, const Win* __restrict__ Sf, const Win* __restrict__ Jf,
                                                     Win* __restrict__ Sc, Win* __restrict__ Jc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * M) return;
  const int c = t % 3;
  const Win sf = Sf[t], jf = Jf[t];
  Win s, jw;
  for (int d = 0; d < 3; ++d) {
    const bool normal = d == c;
    const int bs = sf.base[d];
    s.base[d] = floor_div2(bs);   // lowest coarse face whose stencil reaches fine index bs
    for (int E = 0; E < kW; ++E) {
      const int I = s.base[d] + E;
      double v = 0.0;
      for (int e = 0; e < kW; ++e) {
        const int f = bs + e, dd = f - 2 * I;
        double r = 0.0;
        if (normal) r = dd == 0 ? 0.5 : (dd == 1 || dd == -1) ? 0.25 : 0.0;
        else r = (dd == 0 || dd == 1) ? 0.5 : 0.0;
        v += r * sf.w[d][e];
      }
      s.w[d][E] = v;
    }
    const int bj = jf.base[d];
    jw.base[d] = normal ? floor_div2(bj) : floor_div2(bj) - 1;
    for (int E = 0; E < kW; ++E) {
      const int I = jw.base[d] + E;
      double v = 0.0;
      for (int e = 0; e < kW; ++e) {
        const int f = bj + e, J0 = floor_div2(f);
        const bool even = f - 2 * J0 == 0;
        double pw = 0.0;
        if (normal) pw = even ? (I == J0 ? 1.0 : 0.0) : ((I == J0 || I == J0 + 1) ? 0.5 : 0.0);
        else pw = I == J0 ? 0.75 : (even ? (I == J0 - 1 ? 0.25 : 0.0) : (I == J0 + 1 ? 0.25 : 0.0));
        v += pw * jf.w[d][e];
      }
      jw.w[d][E] = v;
    }
  }
  Sc[t] = s;
  Jc[t] = jw;
}

// ---------------------------------------------------------------- bins and active faces

__global__ void __launch_bounds__(256) k3_bin_count(int M, int N, const Win* __restrict__ S, int* __restrict__ cnt,
                                                    int* __restrict__ key) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * M) return;
  const int c = t % 3;
  const Win& w = S[t];
  const int g = (pmod(w.base[2], N) * N + pmod(w.base[1], N)) * N + pmod(w.base[0], N);
  const int k = c * N * N * N + g;
  key[t] = k;
  atomicAdd(&cnt[k], 1);
}

// Stable placement: a (point, component) goes to its bin at the rank it has
// among the entries of the same key with a smaller index (so each bin lists
// its points in ascending order, independent of scheduling).
__global__ void __launch_bounds__(256) k3_bin_fill(int M, const int* __restrict__ key, const int* __restrict__ start,
                                                   int* __restrict__ pts) {
  __shared__ int sk[1024];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int m3 = 3 * M;
  const int k = t < m3 ? key[t] : -1;
  int rank = 0;
  const int lim = min(m3, (blockIdx.x + 1) * blockDim.x);   // the same for the whole workgroup
  for (int base = 0; base < lim; base += 1024) {   // the keys below lim, 1024 at a time through LDS
    const int n = min(1024, lim - base);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) sk[i] = key[base + i];
    __syncthreads();
    for (int u = 0; u < n; ++u) rank += (base + u < t && sk[u] == k) ? 1 : 0;
  }
  if (t < m3) pts[start[k] + rank] = t / 3;
}

// Faces any S window reaches (per component): flag = 1.
__global__ void __launch_bounds__(256) k3_active_flag(int M, int N, const Win* __restrict__ S, int* __restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * M * kW * kW * kW) return;
  const int pc = t / (kW * kW * kW), e = t - pc * kW * kW * kW;
  const int c = pc % 3;
  const int ex = e % kW, ey = (e / kW) % kW, ez = e / (kW * kW);
  const Win& w = S[pc];
  if (w.w[0][ex] == 0.0 || w.w[1][ey] == 0.0 || w.w[2][ez] == 0.0) return;
  const int g = (pmod(w.base[2] + ez, N) * N + pmod(w.base[1] + ey, N)) * N + pmod(w.base[0] + ex, N);
  flag[c * N * N * N + g] = 1;
}

// Box classes: 1 if a velocity unknown of the box is an active face (the box
// gets its own inverse), else 0; one thread per box.
__global__ void __launch_bounds__(256) k3_box_flags(int N, int n, int nb, const int* __restrict__ act,
                                                    int* __restrict__ boxflag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb * nb * nb) return;
  const int bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
  const int nf = (n + 1) * n * n;
  int hit = 0;   // box_dof of a velocity unknown is also its index in act (component * N^3 + face)
  for (int t = 0; t < 3 * nf && !hit; ++t) hit = act[box_dof(t, bx, by, bz, n, N)];
  boxflag[b] = hit ? 1 : 0;
}

// Exclusive scan in three launches: per-1024 block, block sums, add.
__global__ void __launch_bounds__(1024) k3_scan_block(const int* __restrict__ in, int n, int* __restrict__ out,
                                                      int* __restrict__ bsum) {
  __shared__ int s[1024];
  const int i = blockIdx.x * 1024 + threadIdx.x;
  const int v = i < n ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int a = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

__global__ void __launch_bounds__(1024) k3_scan_sums(int* __restrict__ bsum, int nb, int* __restrict__ total) {
  __shared__ int s[1024];
  int carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int a = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(1024) k3_scan_add(int* __restrict__ out, int n, const int* __restrict__ bsum) {
  const int i = blockIdx.x * 1024 + threadIdx.x;
  if (i < n) out[i] += bsum[blockIdx.x];
}

__global__ void __launch_bounds__(256) k3_compact(const int* __restrict__ flag, const int* __restrict__ pos, int n,
                                                  int* __restrict__ list, int* __restrict__ index) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) list[pos[i]] = i;
  index[i] = flag[i] ? pos[i] : -1;
}

__device__ inline int wave_incl_scan(int v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// CSR of S_l by active face, built once per setup from the bins, one wave
// per face: lane l takes the window offsets l and l + 64 (of 125), pass 0
// counts the entries of each face, pass 1 writes them at the lane's prefix
// (so the order is fixed: by lane, offset, then ascending point in a bin).
template <int kPass>
__global__ void __launch_bounds__(256) k3_csr(Lv3 L, int* __restrict__ count, const int* __restrict__ off,
                                              int* __restrict__ cpt, double* __restrict__ cw) {
  const int lane = threadIdx.x & 63;
  const int q = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (q >= *L.nact) return;   // uniform per wave
  const int N = L.N, N3 = N * N * N;
  const int x = L.act[q], c = x / N3, g = x - c * N3;
  const int i = g % N, j = (g / N) % N, k = g / (N * N);
  int n = 0;
  for (int pass = 0; pass < (kPass ? 2 : 1); ++pass) {
    int w0 = 0;
    if (pass == 1) w0 = off[q] + wave_incl_scan(n, lane) - n;
    int m = 0;
    for (int o = lane; o < kW * kW * kW; o += 64) {
      const int ox = o % kW, oy = (o / kW) % kW, oz = o / (kW * kW);
      const int b = c * N3 + (pmod(k - oz, N) * N + pmod(j - oy, N)) * N + pmod(i - ox, N);
      for (int u = L.bin_start[b]; u < L.bin_start[b + 1]; ++u) {
        const int p = L.bin_pts[u];
        const Win& w = L.S[3 * p + c];
        const double v = w.w[0][ox] * w.w[1][oy] * w.w[2][oz];
        if (v == 0.0) continue;
        if (pass == 1) {
          cpt[w0 + m] = p;
          cw[w0 + m] = v;
        }
        ++m;
      }
    }
    n = m;
  }
  if (!kPass) {
    const int tot = wave_incl_scan(n, lane);
    if (lane == 63) count[q] = tot;
  }
}

// ---------------------------------------------------------------- elastic rows

// U[p, c] = (J_l x_c)(p): one wave per (point, component), lane l taking the
// window entries l and l + 64 of 125, a fixed shuffle tree across lanes.
__global__ void __launch_bounds__(256) k3_gather(Lv3 L, const double* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (t >= 3 * L.M) return;   // uniform per wave
  const int c = t % 3, N = L.N;
  const Win& w = L.J[t];
  const double* xc = x + (size_t)c * N * N * N;
  double s = 0.0;
  for (int e = lane; e < kW * kW * kW; e += 64) {
    const int ex = e % kW, ey = (e / kW) % kW, ez = e / (kW * kW);
    const double wt = w.w[0][ex] * w.w[1][ey] * w.w[2][ez];
    if (wt != 0.0)
      s += wt * xc[(pmod(w.base[2] + ez, N) * N + pmod(w.base[1] + ey, N)) * N + pmod(w.base[0] + ex, N)];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) L.U[t] = s;
}

// F[p, c] = coef (U[prev] - 2 U[p] + U[next])
__global__ void __launch_bounds__(256) k3_force(Lv3 L, double coef, const double* __restrict__ U) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * L.M) return;
  const int p = t / 3, c = t - 3 * p;
  L.F[t] = coef * (U[3 * L.prev[p] + c] - 2.0 * U[t] + U[3 * L.next[p] + c]);
}

// y[c][face] = sum over points of S_l(face, p) F[p, c], active faces only;
// one wave per face, lanes strided over its CSR entries, a fixed reduction
// tree across lanes.
__global__ void __launch_bounds__(256) k3_spread(Lv3 L, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int q = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (q >= *L.nact) return;   // uniform per wave
  const int N3 = L.N * L.N * L.N;
  const int x = L.act[q], c = x / N3;
  double s = 0.0;
  for (int u = L.coff[q] + lane; u < L.coff[q + 1]; u += 64) s += L.cw[u] * L.F[3 * L.cpt[u] + c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) y[x] = s;
}

// r = b - A x (b != null) or r = A x, every unknown of the level; the elastic
// rows come from y (zero off the active faces).
__global__ void __launch_bounds__(256) k3_residual(Lv3 L, const double* __restrict__ b, const double* __restrict__ x,
                                                   double* __restrict__ r, int with_y) {
  const int N = L.N, N3 = N * N * N;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * N3) return;
  const int fam = t / N3, g = t - fam * N3;
  const int i = g % N, j = (g / N) % N, k = g / (N * N);
  const int ip = (k * N + j) * N + ((i + 1) & (N - 1)), im = (k * N + j) * N + ((i - 1) & (N - 1));
  const int jp = (k * N + ((j + 1) & (N - 1))) * N + i, jm = (k * N + ((j - 1) & (N - 1))) * N + i;
  const int kp = (((k + 1) & (N - 1)) * N + j) * N + i, km = (((k - 1) & (N - 1)) * N + j) * N + i;
  double a;
  if (fam < 3) {
    const double* xf = x + (size_t)fam * N3;
    const double* p = x + 3 * (size_t)N3;
    const int back = fam == 0 ? im : fam == 1 ? jm : km;
    a = L.c * xf[g] - L.muh2 * (xf[ip] + xf[im] + xf[jp] + xf[jm] + xf[kp] + xf[km] - 6.0 * xf[g]) +
        L.invh * (p[g] - p[back]);
    if (with_y) a += L.y[t];
  } else {
    a = -L.invh * (x[ip] - x[g] + x[N3 + jp] - x[N3 + g] + x[2 * (size_t)N3 + kp] - x[2 * (size_t)N3 + g]);
  }
  r[t] = b ? b[t] - a : a;
}

// ---------------------------------------------------------------- transfers

__global__ void __launch_bounds__(256) k3_restrict(int Nf, const double* __restrict__ rf, double* __restrict__ rc) {
  const int Nc = Nf / 2, N3c = Nc * Nc * Nc, N3f = Nf * Nf * Nf;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * N3c) return;
  const int fam = t / N3c, g = t - fam * N3c;
  const int I[3] = {g % Nc, (g / Nc) % Nc, g / (Nc * Nc)};
  const double* f = rf + (size_t)fam * N3f;
  double s = 0.0;
  if (fam == 3) {
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) s += f[((2 * I[2] + dz) * Nf + 2 * I[1] + dy) * Nf + 2 * I[0] + dx];
    s *= 0.125;
  } else {
    for (int dz = -1; dz <= 2; ++dz)
      for (int dy = -1; dy <= 2; ++dy)
        for (int dx = -1; dx <= 2; ++dx) {
          const int d[3] = {dx, dy, dz};
          double wgt = 1.0;
          for (int a = 0; a < 3; ++a) {
            if (a == fam) wgt *= d[a] == 0 ? 0.5 : (d[a] == 1 || d[a] == -1) ? 0.25 : 0.0;
            else wgt *= (d[a] == 0 || d[a] == 1) ? 0.5 : 0.0;
          }
          if (wgt == 0.0) continue;
          const int fi = pmod(2 * I[0] + dx, Nf), fj = pmod(2 * I[1] + dy, Nf), fk = pmod(2 * I[2] + dz, Nf);
          s += wgt * f[(fk * Nf + fj) * Nf + fi];
        }
  }
  rc[t] = s;
}

__global__ void __launch_bounds__(256) k3_prolong_add(int Nf, const double* __restrict__ ec, double* __restrict__ wf) {
  const int Nc = Nf / 2, N3c = Nc * Nc * Nc, N3f = Nf * Nf * Nf;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * N3f) return;
  const int fam = t / N3f, g = t - fam * N3f;
  const int f[3] = {g % Nf, (g / Nf) % Nf, g / (Nf * Nf)};
  const double* e = ec + (size_t)fam * N3c;
  if (fam == 3) {
    wf[t] += e[((f[2] / 2) * Nc + f[1] / 2) * Nc + f[0] / 2];
    return;
  }
  int idx[3][2];
  double wt[3][2];
  for (int a = 0; a < 3; ++a) {
    const int J = f[a] / 2;
    const bool even = (f[a] & 1) == 0;
    if (a == fam) {
      idx[a][0] = J; wt[a][0] = even ? 1.0 : 0.5;
      idx[a][1] = J + 1; wt[a][1] = even ? 0.0 : 0.5;
    } else {
      idx[a][0] = J; wt[a][0] = 0.75;
      idx[a][1] = even ? J - 1 : J + 1; wt[a][1] = 0.25;
    }
  }
  double s = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const double wgt = wt[0][cx] * wt[1][cy] * wt[2][cz];
        if (wgt == 0.0) continue;
        s += wgt * e[(pmod(idx[2][cz], Nc) * Nc + pmod(idx[1][cy], Nc)) * Nc + pmod(idx[0][cx], Nc)];
      }
  wf[t] += s;
}

// ---------------------------------------------------------------- box blocks

// sum over the CSR entries (p, S_l(a, p)) of active face a (index ia) of
// S_l(a, p) (J_prev(b) - 2 J_p(b) + J_next(b)): the elastic entry (a, b) of
// component c without the factor -dt K.
__device__ double elastic_entry(const Lv3& L, int c, int ia, int gb) {
  const int N = L.N;
  const int bi = gb % N, bj = (gb / N) % N, bk = gb / (N * N);
  double s = 0.0;
#pragma unroll 4
  for (int u = L.coff[ia]; u < L.coff[ia + 1]; ++u) {
    const int p = L.cpt[u];
    const double jb = wval(L.J[3 * L.prev[p] + c], bi, bj, bk, N) - 2.0 * wval(L.J[3 * p + c], bi, bj, bk, N) +
                      wval(L.J[3 * L.next[p] + c], bi, bj, bk, N);
    s += L.cw[u] * jb;
  }
  return s;
}

// Block of box `boxes[blockIdx.x]` (with the elastic part when with_ib),
// written transposed: out[col][row] = A[row][col].  The elastic entries of a
// velocity row a and column b of component c are coef sum_p S_p(a)
// (J_prev(b) - 2 J_p(b) + J_next(b)) over the CSR entries of row a.
__device__ void box_assemble_body(const Lv3& L, int box, int with_ib, double* __restrict__ B) {
  const int nd = L.nd, n = L.n, N = L.N, nb = L.nb;
  const int bx = box % nb, by = (box / nb) % nb, bz = box / (nb * nb);
  for (int t = threadIdx.x; t < nd * nd; t += blockDim.x) {
    const int col = t / nd, row = t - col * nd;   // B[col][row] = A[row][col]
    B[t] = stokes_entry(L, box_dof(row, bx, by, bz, n, N), box_dof(col, bx, by, bz, n, N));
  }
  if (!with_ib || L.coef == 0.0 || L.M == 0) return;
  __syncthreads();   // the Stokes pass above owns the entries in another order
  const int nf = (n + 1) * n * n, N3 = N * N * N;
  for (int t = threadIdx.x; t < 3 * nf * nf; t += blockDim.x) {
    const int c = t / (nf * nf), rem = t - c * nf * nf;
    const int ra = rem / nf, cb = rem - ra * nf;
    const int ga = box_dof(c * nf + ra, bx, by, bz, n, N) - c * N3;
    const int ia = L.act_index[c * N3 + ga];
    if (ia < 0) continue;
    const int gb = box_dof(c * nf + cb, bx, by, bz, n, N) - c * N3;
    B[(size_t)(c * nf + cb) * nd + c * nf + ra] += L.coef * elastic_entry(L, c, ia, gb);
  }
}

__global__ void __launch_bounds__(kGjThreads) k3_box_assemble(Lv3 L, const int* __restrict__ boxes, int with_ib,
                                                              double* __restrict__ out, size_t stride) {
  box_assemble_body(L, boxes ? boxes[blockIdx.x] : 0, with_ib, out + stride * blockIdx.x);
}

// The boxes with own inverses of all smoothed levels in one launch (the
// levels are independent): workgroup q takes box q - start[l] of level l.
struct OwnJobs {
  Lv3 v[IBMG_MAX_LEVELS];
  int start[IBMG_MAX_LEVELS + 1];
  int nlev;
};

__device__ inline int job_level(const OwnJobs& J, int q) {
  int l = 0;
  while (l + 1 < J.nlev && q >= J.start[l + 1]) ++l;
  return l;
}

// The Stokes part of every own box (one workgroup per box) ...
__global__ void __launch_bounds__(kGjThreads) k3_box_assemble_own(const OwnJobs* __restrict__ J,
                                                                  int* const* __restrict__ own_box,
                                                                  double* const* __restrict__ inv) {
  const int q = blockIdx.x, l = job_level(*J, q), i = q - J->start[l];
  const Lv3& L = J->v[l];
  box_assemble_body(L, own_box[l][i], 0, inv[l] + (size_t)L.nd * L.nd * i);
}

// ... then the elastic entries, one workgroup per (box, component, 16 rows):
// on the coarse levels a face's CSR row holds most of the points, and
// splitting a box fifteen ways keeps those boxes from setting the launch's
// length.  Each entry belongs to one workgroup (stored transposed as above).
constexpr int kElRows = 16;

__global__ void __launch_bounds__(256) k3_box_elastic_own(const OwnJobs* __restrict__ J,
                                                          int* const* __restrict__ own_box,
                                                          double* const* __restrict__ inv) {
  const int q = blockIdx.x, l = job_level(*J, q), i = q - J->start[l];
  const Lv3& L = J->v[l];
  const int n = L.n, N = L.N, nb = L.nb, nd = L.nd, N3 = N * N * N;
  const int nf = (n + 1) * n * n;
  const int c = blockIdx.y / ((nf + kElRows - 1) / kElRows);
  const int r0 = (blockIdx.y - c * ((nf + kElRows - 1) / kElRows)) * kElRows;
  const int box = own_box[l][i];
  const int bx = box % nb, by = (box / nb) % nb, bz = box / (nb * nb);
  double* B = inv[l] + (size_t)nd * nd * i;
  for (int t = threadIdx.x; t < kElRows * nf; t += blockDim.x) {
    const int ra = r0 + t / nf, cb = t % nf;
    if (ra >= nf) break;
    const int ga = box_dof(c * nf + ra, bx, by, bz, n, N) - c * N3;
    const int ia = L.act_index[c * N3 + ga];
    if (ia < 0) continue;
    const int gb = box_dof(c * nf + cb, bx, by, bz, n, N) - c * N3;
    B[(size_t)(c * nf + cb) * nd + c * nf + ra] += L.coef * elastic_entry(L, c, ia, gb);
  }
}

// In-place Gauss-Jordan inverse of each nd x nd matrix, blocked by panels
// of kPanel pivots (no pivoting: the velocity block comes first and has a
// dominant positive diagonal, the pressure pivots are then those of the
// box's Schur complement).  For the pivot block K and the rest R:
//   D = A_KK^{-1};  A_KR <- D A_KR;  A_RR <- A_RR - A_RK A_KR;
//   A_RK <- -A_RK D;  A_KK <- D,
// so the matrix is read and written once per panel instead of once per pivot.
constexpr int kPanel = 8;

__device__ void gj_body(double* __restrict__ A, int nd) {
  __shared__ double rowp[kPanel][kMaxNd];   // rows of K (then D A_KR)
  __shared__ double colp[kMaxNd][kPanel];   // columns of K (A_RK, old)
  __shared__ double dinv[kPanel][kPanel];
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < nd; k0 += kPanel) {
    const int pw = min(kPanel, nd - k0);
    for (int t = tid; t < pw * nd; t += blockDim.x) {
      const int s = t / nd, j = t - s * nd;
      rowp[s][j] = A[(size_t)(k0 + s) * nd + j];
      colp[j][s] = A[(size_t)j * nd + k0 + s];
    }
    __syncthreads();
    if (tid < 64) {   // D = A_KK^{-1}: wave 0, lane (a, b) holds entry (a, b) (identity outside pw)
      const int a = tid >> 3, b = tid & 7;
      double d = (a < pw && b < pw) ? rowp[a][k0 + b] : (a == b ? 1.0 : 0.0);
      for (int k = 0; k < pw; ++k) {
        const double piv = __shfl(d, k * 8 + k);
        const double rk = __shfl(d, k * 8 + b);   // entry (k, b)
        const double ck = __shfl(d, a * 8 + k);   // entry (a, k)
        const double inv = 1.0 / piv;
        if (a == k) d = b == k ? inv : rk * inv;
        else d = b == k ? -ck * inv : d - ck * rk * inv;
      }
      if (a < pw && b < pw) dinv[a][b] = d;
    }
    __syncthreads();
    // new pivot rows D A_KR (columns outside K), one column per thread
    for (int j = tid; j < nd; j += blockDim.x) {
      if (j >= k0 && j < k0 + pw) continue;
      double v[kPanel];
      for (int a = 0; a < pw; ++a) {
        double s = 0.0;
        for (int b = 0; b < pw; ++b) s += dinv[a][b] * rowp[b][j];
        v[a] = s;
      }
      for (int a = 0; a < pw; ++a) rowp[a][j] = v[a];
    }
    __syncthreads();
    // rank-pw update of A_RR and the new blocks: thread (g, j) owns column j
    // for rows g, g + ng, ...; its column of the panel rows sits in
    // registers, the panel column entry colp[i][.] is the same for the lanes
    // of a wave (an LDS broadcast), and the lanes' A accesses are contiguous.
    const int ng = blockDim.x / nd;
    const int g = tid / nd, j = tid - g * nd;
    if (g < ng) {
      const bool jk = j >= k0 && j < k0 + pw;
      double rj[kPanel];
      for (int b = 0; b < kPanel; ++b) rj[b] = b < pw ? (jk ? dinv[b][j - k0] : rowp[b][j]) : 0.0;
      // rows four at a time: the four loads of A are issued before the
      // first product, so each thread keeps four L2 requests in flight
      for (int i0 = g; i0 < nd; i0 += 4 * ng) {
        double a4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r * ng;
          a4[r] = i < nd ? A[(size_t)i * nd + j] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r * ng;
          if (i >= nd) break;
          const bool ik = i >= k0 && i < k0 + pw;
          double v;
          if (ik) {
            v = rj[i - k0];
          } else if (jk) {
            double s = 0.0;
            for (int b = 0; b < pw; ++b) s += colp[i][b] * rj[b];
            v = -s;
          } else {
            double s = a4[r];
            for (int b = 0; b < pw; ++b) s -= colp[i][b] * rj[b];
            v = s;
          }
          A[(size_t)i * nd + j] = v;
        }
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kGjThreads) k3_gj(double* __restrict__ mats, int nd, size_t stride) {
  gj_body(mats + stride * blockIdx.x, nd);
}

__global__ void __launch_bounds__(kGjThreads) k3_gj_own(const OwnJobs* __restrict__ J, double* const* __restrict__ inv) {
  const int q = blockIdx.x, l = job_level(*J, q), i = q - J->start[l];
  const int nd = J->v[l].nd;
  gj_body(inv[l] + (size_t)nd * nd * i, nd);
}

// w[box] += omega A_box^{-1} r[box] for the listed boxes: entry q of the
// list is a box id (plain: shared inverse) or, own, the own index of a box.
// Grid: (boxes / kB, row slices of 64).  In a workgroup each of the eight
// waves takes an eighth of the columns k for the slice's 64 rows (lane =
// row), the partial sums meet in LDS and are added in wave order.
// Plain boxes go kShare to a workgroup so that each load of the shared
// inverse (from L2) serves kShare boxes.
constexpr int kShare = 4;

template <int kB>
__global__ void __launch_bounds__(kBoxThreads) k3_box_apply(Lv3 L, const double* __restrict__ r, double* __restrict__ w,
                                                            const int* __restrict__ list, int count,
                                                            const int* __restrict__ own_box,
                                                            const double* __restrict__ inv, size_t stride) {
  __shared__ double rb[kB][kMaxNd];
  __shared__ double part[kBoxThreads / 64][kB][64];
  const int q0 = blockIdx.x * kB;
  const int nd = L.nd, n = L.n, nb = L.nb;
  const int nbx = min(kB, count - q0);
  int bxs[kB], bys[kB], bzs[kB];
  for (int u = 0; u < kB; ++u) {
    const int id = list[q0 + min(u, nbx - 1)];
    const int box = own_box ? own_box[id] : id;
    bxs[u] = box % nb;
    bys[u] = (box / nb) % nb;
    bzs[u] = box / (nb * nb);
  }
  for (int u = 0; u < kB; ++u)
    for (int t = threadIdx.x; t < nd; t += blockDim.x)
      rb[u][t] = u < nbx ? r[box_dof(t, bxs[u], bys[u], bzs[u], n, L.N)] : 0.0;
  __syncthreads();
  const double* Ai = inv + (own_box ? stride * list[q0] : 0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = blockIdx.y * 64 + lane;
  constexpr int kWaves = kBoxThreads / 64;
  const int kq = (nd + kWaves - 1) / kWaves, k0 = wv * kq, k1 = min(nd, k0 + kq);
  double z[kB];
  for (int u = 0; u < kB; ++u) z[u] = 0.0;
  if (row < nd) {
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
      const double a = Ai[(size_t)k * nd + row];
      for (int u = 0; u < kB; ++u) z[u] += a * rb[u][k];
    }
  }
  for (int u = 0; u < kB; ++u) part[wv][u][lane] = z[u];
  __syncthreads();
  if (wv == 0 && row < nd)
    for (int u = 0; u < nbx; ++u) {
      double v = part[0][u][lane];
      for (int q = 1; q < kWaves; ++q) v += part[q][u][lane];   // wave order
      w[box_dof(row, bxs[u], bys[u], bzs[u], n, L.N)] += L.omega * v;
    }
}

// ---------------------------------------------------------------- coarsest level

// Augmented [B | I] of the bordered coarsest system, one thread per row.
__global__ void __launch_bounds__(256) k3_coarse_assemble(Lv3 L, double* __restrict__ aug, int nr) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nr) return;
  const int N = L.N, N3 = N * N * N, nu = 4 * N3;
  double* a = aug + (size_t)row * 2 * nr;
  for (int col = 0; col < 2 * nr; ++col) a[col] = col - nr == row ? 1.0 : 0.0;
  if (row == nu) {
    for (int col = 3 * N3; col < nu; ++col) a[col] = 1.0;
    return;
  }
  for (int col = 0; col < nu; ++col) a[col] = stokes_entry(L, row, col);
  if (row >= 3 * N3) a[nu] = 1.0;
}

// Elastic entries of the coarsest matrix (after k3_coarse_assemble), NC^3
// cells (NC = 2 or 4): one wave per (component, row a), the lanes strided
// over the CSR entries of row a.  A lane tabulates the per-axis weights of
// its entry's three interpolation windows over the NC coordinates once and
// accumulates every column; the columns are then summed across the lanes by
// a fixed shuffle tree.
template <int NC>
__global__ void __launch_bounds__(64) k3_coarse_elastic(Lv3 L, double* __restrict__ aug, int nr) {
  constexpr int N3 = NC * NC * NC;
  const int lane = threadIdx.x;
  const int c = blockIdx.x / N3, ga = blockIdx.x - c * N3;
  const int ia = L.act_index[c * N3 + ga];
  if (ia < 0) return;
  double acc[N3];
#pragma unroll
  for (int b = 0; b < N3; ++b) acc[b] = 0.0;
  for (int u = L.coff[ia] + lane; u < L.coff[ia + 1]; u += 64) {
    const int p = L.cpt[u];
    const double wa = L.cw[u];
    const int qs[3] = {L.prev[p], p, L.next[p]};
    double tab[3][3][NC];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const Win& Jw = L.J[3 * qs[m] + c];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int x = 0; x < NC; ++x) tab[m][d][x] = wsum(Jw, d, x, NC);
    }
#pragma unroll
    for (int b = 0; b < N3; ++b) {
      const int bi = b % NC, bj = (b / NC) % NC, bk = b / (NC * NC);
      acc[b] += wa * (tab[0][0][bi] * tab[0][1][bj] * tab[0][2][bk] - 2.0 * tab[1][0][bi] * tab[1][1][bj] * tab[1][2][bk] +
                      tab[2][0][bi] * tab[2][1][bj] * tab[2][2][bk]);
    }
  }
#pragma unroll
  for (int b = 0; b < N3; ++b) {
    double v = acc[b];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) aug[(size_t)(c * N3 + ga) * 2 * nr + c * N3 + b] += L.coef * v;
  }
}

// ---------------------------------------------------------------- step pieces

// b = c [u; v; w] + y on the velocity rows (y = S_0 (K L X)), 0 on continuity.
__global__ void __launch_bounds__(256) k3_rhs(int N, double c, const double* __restrict__ uvw,
                                              const double* __restrict__ y, double* __restrict__ b) {
  const int N3 = N * N * N;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * N3) return;
  b[t] = t < 3 * N3 ? c * uvw[t] + (y ? y[t] : 0.0) : 0.0;
}

// Nodal forces K L X into F (the spread pass then forms S_0 F).
__global__ void __launch_bounds__(256) k3_nodal_force(int M, double K, const int* __restrict__ prev,
                                                      const int* __restrict__ next, const double* __restrict__ X,
                                                      double* __restrict__ F) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * M) return;
  const int p = t / 3, c = t - 3 * p;
  F[t] = K * (X[3 * prev[p] + c] - 2.0 * X[t] + X[3 * next[p] + c]);
}

__global__ void __launch_bounds__(256) k3_move(int M, double dt, const double* __restrict__ U, double* __restrict__ X) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 3 * M) X[t] += dt * U[t];
}

__global__ void __launch_bounds__(256) k3_copy(const double* __restrict__ a, double* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void __launch_bounds__(256) k3_axpy(double* __restrict__ x, const double* __restrict__ z, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += z[i];
}

__global__ void __launch_bounds__(256) k3_transpose(const double* __restrict__ a, int nd, double* __restrict__ b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nd * nd) b[(t % nd) * nd + t / nd] = a[t];
}

__global__ void __launch_bounds__(256) k3_finite(const double* __restrict__ x, size_t n, int* __restrict__ bad) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) *bad = 1;
}

}  // namespace

// ---------------------------------------------------------------- handle

struct Lvl3Bufs {
  int N = 0, nb = 0;
  Buf w, b, r, y;
  Buf S, J, key, cnt, start, pts, flag, pos, act, nact, act_index, ccount, coff, cpt, cw;
  Buf boxflag, lists, own_box, inv_plain, inv_own;
  int n_own = 0, max_own = 0;
  int nact_h = 0;                        // active faces (host copy, sets launch sizes)
  int lo[2] = {0, 0}, lc[2] = {0, 0};   // own lists: offset and count per colour
  int po[2] = {0, 0}, pc[2] = {0, 0};   // plain lists
};

struct ibmg3_handle {
  int N = 0, M = 0, nfib = 0, kind = 0, levels = 0, n = 4, nu1 = 1, nu2 = 1, maxit = 100;
  double rho = 1, mu = 1, K = 0, rtol = 1e-8, omega = 1.0, dt = 0.0;
  double plain_dt = 0.0;   // dt of the shared plain-box inverses in the workspace (0: none)
  int nd = 0;
  std::vector<int> prev, next;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  Lvl3Bufs L[IBMG_MAX_LEVELS];
  Buf prev_d, next_d, U, F, bsum, total, bad;
  int nr = 0;
  Buf aug, cm, cpiv, crowpos, cused, cY, cainv;
  Buf V, Z, H, g, cs, sn, y, hc, scal, partial, flags_d, bvec, xvec, yfine;
  Buf jobs, jobptr;             // own-box jobs of all levels (device copies of the two below)
  OwnJobs jobs_h{};             // host sources of the asynchronous copies (kept alive with the handle)
  void* jobptr_h[2 * IBMG_MAX_LEVELS] = {};
  double* flags_h = nullptr;
  bool ready = false;
  template <typename T> T* p(const Buf& b) const { return reinterpret_cast<T*>(ws + b.off); }
  size_t n0() const { return 4 * (size_t)N * N * N; }
};

namespace {

using ibmg::kDotBlocks;
using ibmg::kPW;

void take(size_t& cur, Buf& b, size_t bytes) {
  cur = (cur + 255) & ~(size_t)255;
  b.off = cur;
  b.bytes = bytes;
  cur += std::max<size_t>(bytes, 1);
}

bool has_ib(const ibmg3_handle* h) { return h->M > 0 && h->K != 0.0; }

void layout(ibmg3_handle* h) {
  size_t cur = 0;
  const size_t M = std::max(1, h->M);
  const size_t nd2 = (size_t)h->nd * h->nd;
  for (int l = 0; l < h->levels; ++l) {
    Lvl3Bufs& B = h->L[l];
    B.N = h->N >> l;
    const size_t N3 = (size_t)B.N * B.N * B.N;
    take(cur, B.w, 4 * N3 * sizeof(double));
    take(cur, B.b, 4 * N3 * sizeof(double));
    take(cur, B.r, 4 * N3 * sizeof(double));
    if (has_ib(h)) {
      take(cur, B.y, 3 * N3 * sizeof(double));
      take(cur, B.S, 3 * M * sizeof(Win));
      take(cur, B.J, 3 * M * sizeof(Win));
      take(cur, B.key, 3 * M * sizeof(int));
      take(cur, B.cnt, (3 * N3 + 1) * sizeof(int));
      take(cur, B.start, (3 * N3 + 1) * sizeof(int));
      take(cur, B.pts, 3 * M * sizeof(int));
      take(cur, B.flag, (3 * N3 + 1) * sizeof(int));
      take(cur, B.pos, (3 * N3 + 1) * sizeof(int));
      take(cur, B.act, 3 * N3 * sizeof(int));
      take(cur, B.nact, 4 * sizeof(int));
      take(cur, B.act_index, 3 * N3 * sizeof(int));
      take(cur, B.ccount, (3 * N3 + 1) * sizeof(int));
      take(cur, B.coff, (3 * N3 + 1) * sizeof(int));
      const size_t ent = 3 * M * kW * kW * kW;   // every window entry of every point and component
      take(cur, B.cpt, ent * sizeof(int));
      take(cur, B.cw, ent * sizeof(double));
    }
    if (l < h->levels - 1) {
      B.nb = B.N / h->n;
      const size_t nbox = (size_t)B.nb * B.nb * B.nb;
      take(cur, B.boxflag, nbox * sizeof(int));
      take(cur, B.lists, 2 * nbox * sizeof(int));
      take(cur, B.own_box, nbox * sizeof(int));
      take(cur, B.inv_plain, nd2 * sizeof(double));
      B.max_own = has_ib(h) ? (int)nbox : 0;
      take(cur, B.inv_own, std::max<size_t>(1, (size_t)B.max_own) * nd2 * sizeof(double));
    }
  }
  const size_t N30 = (size_t)h->N * h->N * h->N;
  take(cur, h->prev_d, M * sizeof(int));
  take(cur, h->next_d, M * sizeof(int));
  take(cur, h->U, 3 * M * sizeof(double));
  take(cur, h->F, 3 * M * sizeof(double));
  take(cur, h->bsum, (3 * N30 / 1024 + 4) * sizeof(int));
  take(cur, h->total, 4 * sizeof(int));
  take(cur, h->bad, 4 * sizeof(int));
  const int Nc = h->N >> (h->levels - 1);
  h->nr = 4 * Nc * Nc * Nc + 1;
  const size_t nr = h->nr;
  take(cur, h->aug, nr * 2 * nr * sizeof(double));
  take(cur, h->cm, nr * kPW * sizeof(double));
  take(cur, h->cpiv, nr * sizeof(int));
  take(cur, h->crowpos, nr * sizeof(int));
  take(cur, h->cused, nr * sizeof(int));
  take(cur, h->cY, (size_t)kPW * 2 * nr * sizeof(double));
  take(cur, h->cainv, nr * nr * sizeof(double));
  const size_t n0 = h->n0(), m = h->maxit;
  take(cur, h->V, (m + 1) * n0 * sizeof(double));
  take(cur, h->Z, m * n0 * sizeof(double));
  take(cur, h->H, (m + 1) * (m + 1) * sizeof(double));
  take(cur, h->g, (m + 2) * sizeof(double));
  take(cur, h->cs, (m + 1) * sizeof(double));
  take(cur, h->sn, (m + 1) * sizeof(double));
  take(cur, h->y, (m + 1) * sizeof(double));
  take(cur, h->scal, 16 * sizeof(double));
  take(cur, h->hc, 2 * (m + 2) * sizeof(double));
  // product passes (two vectors per pass) and the update pass's per-workgroup norm shares
  take(cur, h->partial, std::max((size_t)kDotBlocks * 2 * (m + 2), (size_t)nblk(n0)) * sizeof(double));
  take(cur, h->flags_d, 8 * sizeof(double));
  take(cur, h->bvec, n0 * sizeof(double));
  take(cur, h->xvec, n0 * sizeof(double));
  take(cur, h->yfine, 3 * N30 * sizeof(double));
  take(cur, h->jobs, sizeof(OwnJobs));
  take(cur, h->jobptr, 2 * IBMG_MAX_LEVELS * sizeof(void*));
  h->need = cur + 256;
}

Lv3 view(const ibmg3_handle* h, int l) {
  const Lvl3Bufs& B = h->L[l];
  Lv3 v{};
  v.N = B.N;
  v.n = h->n;
  v.nb = B.nb;
  v.nd = h->nd;
  const double hl = 1.0 / B.N;
  v.c = h->rho / h->dt;
  v.muh2 = h->mu / (hl * hl);
  v.invh = 1.0 / hl;
  v.omega = h->omega;
  v.coef = has_ib(h) ? -h->dt * h->K : 0.0;
  v.M = has_ib(h) ? h->M : 0;
  if (has_ib(h)) {
    v.S = h->p<Win>(B.S);
    v.J = h->p<Win>(B.J);
    v.prev = h->p<int>(h->prev_d);
    v.next = h->p<int>(h->next_d);
    v.U = h->p<double>(h->U);
    v.F = h->p<double>(h->F);
    v.bin_start = h->p<int>(B.start);
    v.bin_pts = h->p<int>(B.pts);
    v.act = h->p<int>(B.act);
    v.nact = h->p<int>(B.nact);
    v.act_index = h->p<int>(B.act_index);
    v.coff = h->p<int>(B.coff);
    v.cpt = h->p<int>(B.cpt);
    v.cw = h->p<double>(B.cw);
    v.y = h->p<double>(B.y);
  }
  return v;
}

template <typename T> void fill(hipStream_t s, T* x, size_t n, T v) {
  k_fill<T><<<nblk(n), 256, 0, s>>>(x, n, v);
}

// Exclusive scan of n ints into out; the sum of all n into h->total.
void scan(ibmg3_handle* h, const int* in, int n, int* out) {
  hipStream_t s = h->stream;
  const int nb = (n + 1023) / 1024;
  k3_scan_block<<<nb, 1024, 0, s>>>(in, n, out, h->p<int>(h->bsum));
  k3_scan_sums<<<1, 1024, 0, s>>>(h->p<int>(h->bsum), nb, h->p<int>(h->total));
  k3_scan_add<<<nb, 1024, 0, s>>>(out, n, h->p<int>(h->bsum));
}

// Elastic rows y_l = M_l x (into the level's y), or nothing without structure.
void elastic_rows(ibmg3_handle* h, int l, const double* x) {
  if (!has_ib(h)) return;
  hipStream_t s = h->stream;
  Lv3 v = view(h, l);
  const int m3 = 3 * h->M;
  k3_gather<<<nblk((size_t)m3 * 64), 256, 0, s>>>(v, x);
  k3_force<<<nblk(m3), 256, 0, s>>>(v, v.coef, v.U);
  if (h->L[l].nact_h > 0) k3_spread<<<nblk((size_t)h->L[l].nact_h * 64), 256, 0, s>>>(v, v.y);
}

void residual(ibmg3_handle* h, int l, const double* b, const double* x, double* r) {
  elastic_rows(h, l, x);
  Lv3 v = view(h, l);
  const size_t N3 = (size_t)v.N * v.N * v.N;
  k3_residual<<<nblk(4 * N3), 256, 0, h->stream>>>(v, b, x, r, has_ib(h) ? 1 : 0);
}

void sweep(ibmg3_handle* h, int l, const double* b, double* w) {
  hipStream_t s = h->stream;
  Lvl3Bufs& B = h->L[l];
  Lv3 v = view(h, l);
  double* r = h->p<double>(B.r);
  const int* lists = h->p<int>(B.lists);
  for (int c = 0; c < 2; ++c) {
    residual(h, l, b, w, r);
    const unsigned slices = (unsigned)((h->nd + 63) / 64);
    if (B.lc[c] > 0)
      k3_box_apply<1><<<dim3(B.lc[c], slices), kBoxThreads, 0, s>>>(v, r, w, lists + B.lo[c], B.lc[c],
                                                                    h->p<int>(B.own_box), h->p<double>(B.inv_own),
                                                                    (size_t)h->nd * h->nd);
    if (B.pc[c] > 0)
      k3_box_apply<kShare><<<dim3((B.pc[c] + kShare - 1) / kShare, slices), kBoxThreads, 0, s>>>(
          v, r, w, lists + B.po[c], B.pc[c], nullptr, h->p<double>(B.inv_plain), 0);
  }
}

void vcycle_level(ibmg3_handle* h, int l, const double* b, double* w) {
  hipStream_t s = h->stream;
  const size_t N3 = (size_t)h->L[l].N * h->L[l].N * h->L[l].N;
  if (l == h->levels - 1) {
    ibmg::launch_coarse_apply<double>(s, h->p<double>(h->cainv), h->nr, b, w);
    return;
  }
  fill<double>(s, w, 4 * N3, 0.0);
  for (int q = 0; q < h->nu1; ++q) sweep(h, l, b, w);
  double* r = h->p<double>(h->L[l].r);
  residual(h, l, b, w, r);
  Lvl3Bufs& C = h->L[l + 1];
  k3_restrict<<<nblk(4 * (N3 / 8)), 256, 0, s>>>(h->L[l].N, r, h->p<double>(C.b));
  vcycle_level(h, l + 1, h->p<double>(C.b), h->p<double>(C.w));
  k3_prolong_add<<<nblk(4 * N3), 256, 0, s>>>(h->L[l].N, h->p<double>(C.w), w);
  for (int q = 0; q < h->nu2; ++q) sweep(h, l, b, w);
}

int sync(ibmg3_handle* h) {
  return hipStreamSynchronize(h->stream) == hipSuccess ? IBMG_OK : IBMG_EHIP;
}

int read_doubles(ibmg3_handle* h, const double* d, double* out, int n) {
  IBMG_HIP(hipMemcpyAsync(h->flags_h, d, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  IBMG_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < n; ++i) out[i] = reinterpret_cast<volatile double*>(h->flags_h)[i];
  return IBMG_OK;
}

void dot(ibmg3_handle* h, const double* a, const double* b, double* out) {
  ibmg::launch_multidot(h->stream, a, 0, 1, b, h->n0(), h->p<double>(h->partial), kDotBlocks);
  ibmg::launch_reduce(h->stream, h->p<double>(h->partial), kDotBlocks, 1, out, 0);
}

int build_level(ibmg3_handle* h, int l) {
  hipStream_t s = h->stream;
  Lvl3Bufs& B = h->L[l];
  const int N = B.N;
  const size_t N3 = (size_t)N * N * N;
  const int m3 = 3 * h->M;
  if (has_ib(h)) {
    if (l > 0)
      k3_win_coarse<<<nblk(m3), 256, 0, s>>>(h->M, h->p<Win>(h->L[l - 1].S), h->p<Win>(h->L[l - 1].J),
                                            h->p<Win>(B.S), h->p<Win>(B.J));
    fill<int>(s, h->p<int>(B.cnt), 3 * N3 + 1, 0);
    k3_bin_count<<<nblk(m3), 256, 0, s>>>(h->M, N, h->p<Win>(B.S), h->p<int>(B.cnt), h->p<int>(B.key));
    scan(h, h->p<int>(B.cnt), (int)(3 * N3 + 1), h->p<int>(B.start));
    k3_bin_fill<<<nblk(m3), 256, 0, s>>>(h->M, h->p<int>(B.key), h->p<int>(B.start), h->p<int>(B.pts));
    fill<int>(s, h->p<int>(B.flag), 3 * N3 + 1, 0);
    k3_active_flag<<<nblk((size_t)m3 * kW * kW * kW), 256, 0, s>>>(h->M, N, h->p<Win>(B.S), h->p<int>(B.flag));
    scan(h, h->p<int>(B.flag), (int)(3 * N3 + 1), h->p<int>(B.pos));
    k3_compact<<<nblk(3 * N3), 256, 0, s>>>(h->p<int>(B.flag), h->p<int>(B.pos), (int)(3 * N3), h->p<int>(B.act),
                                            h->p<int>(B.act_index));
    IBMG_HIP(hipMemcpyAsync(h->p<int>(B.nact), h->p<int>(h->total), sizeof(int), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(&B.nact_h, h->p<int>(h->total), sizeof(int), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    if (B.nact_h > 0) {
      Lv3 v = view(h, l);
      const unsigned blocks = nblk((size_t)B.nact_h * 64);
      fill<int>(s, h->p<int>(B.ccount), 3 * N3 + 1, 0);
      k3_csr<0><<<blocks, 256, 0, s>>>(v, h->p<int>(B.ccount), nullptr, nullptr, nullptr);
      scan(h, h->p<int>(B.ccount), (int)(3 * N3 + 1), h->p<int>(B.coff));
      k3_csr<1><<<blocks, 256, 0, s>>>(v, nullptr, h->p<int>(B.coff), h->p<int>(B.cpt), h->p<double>(B.cw));
    }
    fill<double>(s, h->p<double>(B.y), 3 * N3, 0.0);
  }
  if (l == h->levels - 1) return IBMG_OK;
  // box classes: own (a velocity unknown of the box is an active face) or plain
  const int nb = B.nb;
  const int nbox = nb * nb * nb;
  std::vector<int> flag(nbox, 0);
  if (has_ib(h)) {
    k3_box_flags<<<nblk(nbox), 256, 0, s>>>(N, h->n, nb, h->p<int>(B.flag), h->p<int>(B.boxflag));
    IBMG_HIP(hipMemcpyAsync(flag.data(), h->p<int>(B.boxflag), nbox * sizeof(int), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
  }
  std::vector<int> lists, own_box;
  int nown = 0;
  for (int c = 0; c < 2; ++c) {
    B.lo[c] = (int)lists.size();
    for (int b = 0; b < nbox; ++b) {
      const int bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
      if ((bx + by + bz) % 2 == c && flag[b]) {
        lists.push_back(nown++);
        own_box.push_back(b);
      }
    }
    B.lc[c] = (int)lists.size() - B.lo[c];
    B.po[c] = (int)lists.size();
    for (int b = 0; b < nbox; ++b) {
      const int bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
      if ((bx + by + bz) % 2 == c && !flag[b]) lists.push_back(b);
    }
    B.pc[c] = (int)lists.size() - B.po[c];
  }
  B.n_own = nown;
  if (nown > B.max_own) return IBMG_ENOMEM;
  IBMG_HIP(hipMemcpyAsync(h->p<int>(B.lists), lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (nown)
    IBMG_HIP(hipMemcpyAsync(h->p<int>(B.own_box), own_box.data(), nown * sizeof(int), hipMemcpyHostToDevice, s));
  // the host vectors are read by the copies: wait before they go out of scope
  IBMG_HIP(hipStreamSynchronize(s));
  Lv3 v = view(h, l);
  const size_t nd2 = (size_t)h->nd * h->nd;
  if (h->plain_dt != h->dt) {   // the plain block depends on rho / dt, mu and h only
    k3_box_assemble<<<1, kGjThreads, 0, s>>>(v, nullptr, 0, h->p<double>(B.inv_plain), nd2);
    k3_gj<<<1, kGjThreads, 0, s>>>(h->p<double>(B.inv_plain), h->nd, nd2);
  }
  return IBMG_OK;
}

int do_setup(ibmg3_handle* h, double dt, const double* X) {
  if (!h->ws) return IBMG_ESTATE;
  if (!(dt > 0) || !std::isfinite(dt)) return IBMG_EINVAL;
  if (has_ib(h) && !X) return IBMG_EINVAL;
  hipStream_t s = h->stream;
  h->dt = dt;
  h->ready = false;
  if (has_ib(h)) {
    int* bad = h->p<int>(h->bad);
    fill<int>(s, bad, 1, 0);
    k3_finite<<<nblk(3 * (size_t)h->M), 256, 0, s>>>(X, 3 * (size_t)h->M, bad);
    int hb = 0;
    IBMG_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    if (hb) return IBMG_ENONFINITE;
    k3_win0<<<nblk(3 * (size_t)h->M), 256, 0, s>>>(h->M, h->N, h->kind, X, h->p<Win>(h->L[0].S),
                                                 h->p<Win>(h->L[0].J));
  }
  for (int l = 0; l < h->levels; ++l) {
    const int rc = build_level(h, l);
    if (rc) {
      h->plain_dt = 0.0;
      return rc;
    }
  }
  h->plain_dt = h->dt;
  // the boxes with own inverses of every smoothed level: one assembly and
  // one Gauss-Jordan launch for all levels
  {
    OwnJobs& J = h->jobs_h;
    int total = 0;
    J.nlev = h->levels - 1;
    for (int l = 0; l < J.nlev; ++l) {
      J.v[l] = view(h, l);
      J.start[l] = total;
      total += h->L[l].n_own;
      h->jobptr_h[l] = h->p<int>(h->L[l].own_box);
      h->jobptr_h[IBMG_MAX_LEVELS + l] = h->p<double>(h->L[l].inv_own);
    }
    J.start[J.nlev] = total;
    if (total > 0) {
      IBMG_HIP(hipMemcpyAsync(h->p<OwnJobs>(h->jobs), &J, sizeof(OwnJobs), hipMemcpyHostToDevice, s));
      IBMG_HIP(hipMemcpyAsync(h->p<void*>(h->jobptr), h->jobptr_h, sizeof(h->jobptr_h), hipMemcpyHostToDevice, s));
      int* const* boxes = reinterpret_cast<int* const*>(h->p<void*>(h->jobptr));
      double* const* invs = reinterpret_cast<double* const*>(h->p<void*>(h->jobptr) + IBMG_MAX_LEVELS);
      k3_box_assemble_own<<<total, kGjThreads, 0, s>>>(h->p<OwnJobs>(h->jobs), boxes, invs);
      const int nf = (h->n + 1) * h->n * h->n;
      k3_box_elastic_own<<<dim3(total, 3 * ((nf + kElRows - 1) / kElRows)), 256, 0, s>>>(h->p<OwnJobs>(h->jobs),
                                                                                       boxes, invs);
      k3_gj_own<<<total, kGjThreads, 0, s>>>(h->p<OwnJobs>(h->jobs), invs);
    }
  }
  Lv3 vc = view(h, h->levels - 1);
  k3_coarse_assemble<<<nblk(h->nr), 256, 0, s>>>(vc, h->p<double>(h->aug), h->nr);
  if (has_ib(h)) {
    const size_t N3c = (size_t)vc.N * vc.N * vc.N;
    if (vc.N == 4) k3_coarse_elastic<4><<<(unsigned)(3 * N3c), 64, 0, s>>>(vc, h->p<double>(h->aug), h->nr);
    else k3_coarse_elastic<2><<<(unsigned)(3 * N3c), 64, 0, s>>>(vc, h->p<double>(h->aug), h->nr);
  }
  if (ibmg::coarse_factor(s, h->p<double>(h->aug), h->nr, h->p<double>(h->cm), h->p<int>(h->cpiv), nullptr,
                          h->p<int>(h->crowpos), h->p<int>(h->cused), h->p<double>(h->cY),
                          h->p<double>(h->cainv)) != 0)
    return IBMG_EHIP;
  const int rc = sync(h);
  if (rc) return rc;
  h->ready = true;
  return IBMG_OK;
}

int do_solve(ibmg3_handle* h, const double* b, double* x, ibmg_stats* st) {
  hipStream_t s = h->stream;
  const size_t n0 = h->n0();
  const int m = h->maxit, ldh = m + 1;
  double* V = h->p<double>(h->V);
  double* Z = h->p<double>(h->Z);
  double* H = h->p<double>(h->H);
  double* g = h->p<double>(h->g);
  double* scal = h->p<double>(h->scal);
  double* partial = h->p<double>(h->partial);
  double* hc = h->p<double>(h->hc);
  double* cs = h->p<double>(h->cs);
  double* sn = h->p<double>(h->sn);
  double* flags = h->p<double>(h->flags_d);
  double hs[4];
  st->iters = 0;
  st->converged = 0;
  st->fallback = 0;
  dot(h, b, b, scal);
  int rc = read_doubles(h, scal, hs, 1);
  if (rc) return rc;
  const double bnorm = std::sqrt(hs[0]);
  if (!std::isfinite(bnorm)) return IBMG_ENONFINITE;
  st->bnorm = bnorm;
  if (bnorm == 0.0) {
    fill<double>(s, x, n0, 0.0);
    st->converged = 1;
    return sync(h);
  }
  const double target = h->rtol * bnorm;
  residual(h, 0, b, x, V);
  dot(h, V, V, scal);
  if ((rc = read_doubles(h, scal, hs, 1))) return rc;
  const double beta = std::sqrt(hs[0]);
  if (!std::isfinite(beta)) return IBMG_ENONFINITE;
  st->rel_resid_true = st->rel_resid_est = beta / bnorm;
  if (beta <= target) {
    st->converged = 1;
    return IBMG_OK;
  }
  ibmg::launch_scale(s, V, V, n0, scal);
  fill<double>(s, g, m + 2, 0.0);
  fill<double>(s, H, (size_t)(m + 1) * (m + 1), 0.0);
  IBMG_HIP(hipMemcpyAsync(g, &beta, sizeof(double), hipMemcpyHostToDevice, s));
  int k = 0;
  for (int j = 0; j < m; ++j) {
    double* vj = V + (size_t)j * n0;
    double* vn = V + (size_t)(j + 1) * n0;
    double* zj = Z + (size_t)j * n0;
    double* colj = H + (size_t)j * ldh;
    vcycle_level(h, 0, vj, zj);
    residual(h, 0, nullptr, zj, vn);
    // delayed classical Gram-Schmidt (the low-synchronisation DCGS2 form of
    // the 2-D solver): one pass forms the products of the basis with u_j and
    // w, it completes u_j into v_j, column j - 1 and projects w; the
    // stopping test uses column j before its delayed projection
    ibmg::launch_multidot2(s, V, n0, j + 1, vj, vn, n0, partial, kDotBlocks);
    ibmg::launch_reduce(s, partial, kDotBlocks, 2 * (j + 1), hc, 0);
    ibmg::launch_dcgs2_coef(s, hc, hc + (j + 1), j - 1, H, ldh, cs, sn, g, scal + 2);
    ibmg::launch_dcgs2_update(s, V, n0, j, hc, hc + (j + 1), scal + 2, n0, partial);
    ibmg::launch_reduce2(s, partial, (int)nblk(n0), colj + j + 1, scal + 1);
    ibmg::launch_scale_tentative(s, vn, n0, scal + 1, H, ldh, g, cs, sn, j, flags, target);
    if ((rc = read_doubles(h, flags, hs, 3))) return rc;
    k = j + 1;
    st->rel_resid_est = hs[0] / bnorm;
    if (hs[2] != 0.0) return IBMG_ENONFINITE;
    if (hs[1] != 0.0) break;
  }
  if (k > 0) {   // complete column k - 1 (second projection of u_k)
    const int c = k - 1;
    ibmg::launch_multidot(s, V, n0, c + 2, V + (size_t)(c + 1) * n0, n0, partial, kDotBlocks);
    ibmg::launch_reduce(s, partial, kDotBlocks, c + 2, hc, 0);
    ibmg::launch_dcgs2_coef(s, hc, nullptr, c, H, ldh, cs, sn, g, scal + 2);
  }
  ibmg::launch_backsolve(s, H, ldh, g, k, h->p<double>(h->y));
  ibmg::launch_update(s, Z, n0, k, h->p<double>(h->y), x, n0, 1.0);
  st->iters = k;
  double* rt = h->p<double>(h->L[0].r);
  residual(h, 0, b, x, rt);
  dot(h, rt, rt, scal);
  if ((rc = read_doubles(h, scal, hs, 1))) return rc;
  st->rel_resid_true = std::sqrt(hs[0]) / bnorm;
  st->converged = st->rel_resid_true <= h->rtol;
  return st->converged ? IBMG_OK : IBMG_NOT_CONVERGED;
}

// S_0 (K L X) on the velocity faces (zero off the active faces), with the
// level-0 windows of the last setup.
const double* spread_nodal_force(ibmg3_handle* h, const double* X) {
  hipStream_t s = h->stream;
  Lv3 v = view(h, 0);
  const size_t N3 = (size_t)h->N * h->N * h->N;
  double* y = h->p<double>(h->yfine);
  fill<double>(s, y, 3 * N3, 0.0);
  k3_nodal_force<<<nblk(3 * (size_t)h->M), 256, 0, s>>>(h->M, h->K, v.prev, v.next, X, v.F);
  if (h->L[0].nact_h > 0) k3_spread<<<nblk((size_t)h->L[0].nact_h * 64), 256, 0, s>>>(v, y);
  return y;
}

int check_level(const ibmg3_handle* h, int l, bool smoothed) {
  if (!h || !h->ready) return IBMG_ESTATE;
  if (l < 0 || l >= h->levels || (smoothed && l == h->levels - 1)) return IBMG_EINVAL;
  return IBMG_OK;
}

}  // namespace

extern "C" {

int ibmg3_create(ibmg3_handle** out, const ibmg3_problem* pr, const ibmg3_opts* op, void* stream) {
  if (!out || !pr || !op) return IBMG_EINVAL;
  *out = nullptr;
  const int N = pr->N;
  if (N < 8 || N > 128 || (N & (N - 1))) return IBMG_EINVAL;
  if (!(pr->rho > 0) || !(pr->mu > 0) || !std::isfinite(pr->K) || pr->K < 0) return IBMG_EINVAL;
  if (pr->delta != IBMG_DELTA_IB4 && pr->delta != IBMG_DELTA_COS4) return IBMG_EINVAL;
  if (pr->M < 0 || pr->nfib < 0 || (pr->M > 0 && (pr->nfib < 1 || !pr->fiber_offsets))) return IBMG_EINVAL;
  if (op->box != 2 && op->box != 4) return IBMG_EINVAL;
  if (op->levels < 2 || op->levels > IBMG_MAX_LEVELS) return IBMG_EINVAL;
  const int Nc = N >> (op->levels - 1);
  if (Nc < 2 || Nc > 4) return IBMG_EINVAL;   // bordered coarsest system of at most 257 unknowns
  for (int l = 0; l + 1 < op->levels; ++l) {
    const int Nl = N >> l;
    if (Nl % op->box || (Nl / op->box) % 2) return IBMG_EINVAL;
  }
  if (op->nu1 < 0 || op->nu1 > 8 || op->nu2 < 0 || op->nu2 > 8 || op->nu1 + op->nu2 == 0) return IBMG_EINVAL;
  if (op->maxit < 1 || op->maxit > 500 || !(op->rtol > 0) || !(op->omega > 0) || op->omega > 1) return IBMG_EINVAL;
  ibmg3_handle* h = new (std::nothrow) ibmg3_handle();
  if (!h) return IBMG_ENOMEM;
  h->N = N;
  h->M = pr->M;
  h->nfib = pr->nfib;
  h->kind = pr->delta;
  h->rho = pr->rho;
  h->mu = pr->mu;
  h->K = pr->K;
  h->levels = op->levels;
  h->n = op->box;
  h->nu1 = op->nu1;
  h->nu2 = op->nu2;
  h->maxit = op->maxit;
  h->rtol = op->rtol;
  h->omega = op->omega;
  h->nd = 3 * (h->n + 1) * h->n * h->n + h->n * h->n * h->n;
  h->stream = (hipStream_t)stream;
  if (h->M > 0) {
    const int* o = pr->fiber_offsets;
    bool ok = o[0] == 0 && o[h->nfib] == h->M;
    for (int f = 0; f < h->nfib && ok; ++f) ok = o[f + 1] - o[f] >= 3 && o[f + 1] <= h->M;
    if (!ok) {
      delete h;
      return IBMG_EINVAL;
    }
    h->prev.resize(h->M);
    h->next.resize(h->M);
    for (int f = 0; f < h->nfib; ++f) {
      const int a = o[f], b = o[f + 1], len = b - a;
      if (len < 3) {
        delete h;
        return IBMG_EINVAL;
      }
      for (int q = a; q < b; ++q) {
        h->prev[q] = a + (q - a - 1 + len) % len;
        h->next[q] = a + (q - a + 1) % len;
      }
    }
  }
  layout(h);
  *out = h;
  return IBMG_OK;
}

int ibmg3_workspace_bytes(const ibmg3_handle* h, size_t* bytes) {
  if (!h || !bytes) return IBMG_EINVAL;
  *bytes = h->need;
  return IBMG_OK;
}

int ibmg3_bind_workspace(ibmg3_handle* h, void* dev, size_t bytes) {
  if (!h || !dev) return IBMG_EINVAL;
  if (bytes < h->need || (reinterpret_cast<uintptr_t>(dev) & 255)) return IBMG_ENOMEM;
  if (!h->flags_h && hipHostMalloc((void**)&h->flags_h, 64, hipHostMallocDefault) != hipSuccess) return IBMG_EHIP;
  h->ws = (char*)dev;
  h->ws_bytes = bytes;
  h->ready = false;
  h->plain_dt = 0.0;
  if (h->M > 0) {
    IBMG_HIP(hipMemcpyAsync(h->p<int>(h->prev_d), h->prev.data(), h->M * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
    IBMG_HIP(hipMemcpyAsync(h->p<int>(h->next_d), h->next.data(), h->M * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
    IBMG_HIP(hipStreamSynchronize(h->stream));
  }
  return IBMG_OK;
}

int ibmg3_destroy(ibmg3_handle* h) {
  if (!h) return IBMG_EINVAL;
  if (h->flags_h) (void)hipHostFree(h->flags_h);
  delete h;
  return IBMG_OK;
}

int ibmg3_setup(ibmg3_handle* h, double dt, const double* X) {
  if (!h) return IBMG_EINVAL;
  return do_setup(h, dt, X);
}

int ibmg3_apply(ibmg3_handle* h, int32_t level, const double* x, double* y) {
  int rc = check_level(h, level, false);
  if (rc) return rc;
  if (!x || !y) return IBMG_EINVAL;
  residual(h, level, nullptr, x, y);
  return sync(h);
}

int ibmg3_restrict(ibmg3_handle* h, int32_t level, const double* rf, double* rc_) {
  int rc = check_level(h, level, true);
  if (rc) return rc;
  if (!rf || !rc_) return IBMG_EINVAL;
  const size_t Nc = h->L[level + 1].N;
  k3_restrict<<<nblk(4 * Nc * Nc * Nc), 256, 0, h->stream>>>(h->L[level].N, rf, rc_);
  return sync(h);
}

int ibmg3_prolong_add(ibmg3_handle* h, int32_t level, const double* ec, double* wf) {
  int rc = check_level(h, level, true);
  if (rc) return rc;
  if (!ec || !wf) return IBMG_EINVAL;
  const size_t Nf = h->L[level].N;
  k3_prolong_add<<<nblk(4 * Nf * Nf * Nf), 256, 0, h->stream>>>((int)Nf, ec, wf);
  return sync(h);
}

int ibmg3_box_matrix(ibmg3_handle* h, int32_t level, int32_t bx, int32_t by, int32_t bz, double* out) {
  int rc = check_level(h, level, true);
  if (rc) return rc;
  const int nb = h->L[level].nb;
  if (!out || bx < 0 || by < 0 || bz < 0 || bx >= nb || by >= nb || bz >= nb) return IBMG_EINVAL;
  hipStream_t s = h->stream;
  const int box = (bz * nb + by) * nb + bx;
  int* slot = h->p<int>(h->total) + 1;
  IBMG_HIP(hipMemcpyAsync(slot, &box, sizeof(int), hipMemcpyHostToDevice, s));
  double* tmp = h->p<double>(h->V);   // basis storage, free outside a solve
  k3_box_assemble<<<1, kGjThreads, 0, s>>>(view(h, level), slot, 1, tmp, 0);
  k3_transpose<<<nblk((size_t)h->nd * h->nd), 256, 0, s>>>(tmp, h->nd, out);
  return sync(h);
}

int ibmg3_smooth(ibmg3_handle* h, int32_t level, const double* b, double* w, int32_t sweeps) {
  int rc = check_level(h, level, true);
  if (rc) return rc;
  if (!b || !w || sweeps < 0) return IBMG_EINVAL;
  for (int q = 0; q < sweeps; ++q) sweep(h, level, b, w);
  return sync(h);
}

int ibmg3_vcycle(ibmg3_handle* h, const double* r, double* z) {
  int rc = check_level(h, 0, false);
  if (rc) return rc;
  if (!r || !z) return IBMG_EINVAL;
  vcycle_level(h, 0, r, z);
  return sync(h);
}

int ibmg3_rhs(ibmg3_handle* h, const double* uvw, const double* X, double* b) {
  int rc = check_level(h, 0, false);
  if (rc) return rc;
  if (!uvw || !b || (has_ib(h) && !X)) return IBMG_EINVAL;
  hipStream_t s = h->stream;
  const size_t N3 = (size_t)h->N * h->N * h->N;
  const double* y = has_ib(h) ? spread_nodal_force(h, X) : nullptr;
  k3_rhs<<<nblk(4 * N3), 256, 0, s>>>(h->N, h->rho / h->dt, uvw, y, b);
  return sync(h);
}

int ibmg3_solve(ibmg3_handle* h, const double* b, double* x, ibmg_stats* st) {
  int rc = check_level(h, 0, false);
  if (rc) return rc;
  if (!b || !x) return IBMG_EINVAL;
  ibmg_stats tmp{};
  ibmg_stats* s = st ? st : &tmp;
  *s = ibmg_stats{};
  return do_solve(h, b, x, s);
}

int ibmg3_step(ibmg3_handle* h, double dt, double* uvw, double* p, double* X, ibmg_stats* st) {
  if (!h || !uvw || !p || (has_ib(h) && !X)) return IBMG_EINVAL;
  ibmg_stats tmp{};
  ibmg_stats* so = st ? st : &tmp;
  *so = ibmg_stats{};
  int rc = do_setup(h, dt, X);
  if (rc) return rc;
  hipStream_t s = h->stream;
  const size_t N3 = (size_t)h->N * h->N * h->N, n0 = h->n0();
  double* b = h->p<double>(h->bvec);
  double* x = h->p<double>(h->xvec);
  const double* y = nullptr;
  if (has_ib(h)) y = spread_nodal_force(h, X);
  k3_rhs<<<nblk(n0), 256, 0, s>>>(h->N, h->rho / dt, uvw, y, b);
  k3_copy<<<nblk(3 * N3), 256, 0, s>>>(uvw, x, 3 * N3);
  k3_copy<<<nblk(N3), 256, 0, s>>>(p, x + 3 * N3, N3);
  rc = do_solve(h, b, x, so);
  if (rc < 0) return rc;
  const int conv = rc;
  k3_copy<<<nblk(3 * N3), 256, 0, s>>>(x, uvw, 3 * N3);
  k3_copy<<<nblk(N3), 256, 0, s>>>(x + 3 * N3, p, N3);
  if (has_ib(h)) {
    Lv3 v = view(h, 0);
    k3_gather<<<nblk(3 * (size_t)h->M * 64), 256, 0, s>>>(v, uvw);
    k3_move<<<nblk(3 * (size_t)h->M), 256, 0, s>>>(h->M, dt, v.U, X);
  }
  rc = sync(h);
  return rc ? rc : conv;
}

int ibmg3_box_counts(const ibmg3_handle* h, int32_t level, int32_t* own, int32_t* total) {
  int rc = check_level(h, level, true);
  if (rc) return rc;
  if (own) *own = h->L[level].n_own;
  if (total) *total = h->L[level].nb * h->L[level].nb * h->L[level].nb;
  return IBMG_OK;
}

}  // extern "C"
