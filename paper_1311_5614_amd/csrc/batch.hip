// Batched form: many independent implicit IB problems of different grid and
// structure sizes advanced together.  Each problem keeps its own handle
// (workspace, setup, operators), and the solve runs all problems in lockstep
// FGMRES rounds: every V-cycle step and every Krylov step is one launch over
// all problems that take part in it.  The kernels call the same device
// bodies as the single-problem kernels on the same data, with the same
// per-problem block decomposition, so each problem's result is bitwise
// equal to a single-problem run with the same options.
//
// V-cycle (Algorithm 1, Sec. 3): the levels of every problem are aligned
// from the bottom -- step k of the descent is the level whose size is
// 2^(k+1) times the first LDS-resident level -- so one launch covers the
// k-th level of every problem that has it.  The level kernels are
// persistent: a fixed grid drains the (problem, block) list of its step,
// built on the device from the round's active mask, so the whole V-cycle is
// captured once into a hipGraph and replayed however the active set changes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ibmg.h"
#include "common.h"
#include "handle.h"
#include "kernels.h"
#include "level_ops.h"

namespace {

using namespace ibmg;

constexpr int kWorkStreams = 4;  // concurrent streams for the per-problem setup (hardware queues per process)
constexpr int kCap256 = 2048;   // persistent grid of the 256-lane level kernels (8 per CU)
constexpr int kCapBox = 8192;   // persistent grid of the 64-lane box kernel (32 per CU)
constexpr int kCapBox8 = 2048;  // persistent grid of the 256-lane 8 x 8 box kernel (8 per CU)

enum { OP_FILL0 = 0, OP_RES, OP_BOX, OP_BOX8, OP_RESID, OP_RESTRICT, OP_PROLONG, OP_TAIL };

// One problem's level in a batched V-cycle step.
template <typename T>
struct BLv {
  LevelView<T> L;
  const T* b;
  T* w;
  T* r;
  T* bc;      // next coarser level: right-hand side and iterate
  T* wc;
  int nres;   // residual workgroups (3 N_l^2 / 256)
  int nibr;   // elastic-row workgroups of the fused residual (both components)
};

// Per-problem Krylov state (FP64).
struct BKry {
  LevelView<double> v0;
  const double* b;
  double* x;
  double *V, *Z, *H, *g, *cs, *sn, *y, *flags, *scal, *hc, *partial;
  void* b0;
  void* w0;
  long long n0;
  int ldh, m, nibx, pad;
  double target;
};

// A set of problems taking part in one Krylov step of a round.
struct BSet {
  int n;                  // slots
  const int* p;           // problem of each slot
  const int* j;           // inner index (or k for the final update)
  const int* off;         // prefix of element workgroups (3 N^2 / 256 per problem)
  const int* off2;        // prefix of elastic-row workgroups
  const double* beta;     // initial residual norm of each slot
};

// XCD-aware order of a launch's work items: with workgroups dispatched to
// the eight XCDs round-robin, item t is taken as item xcd_order(t, total) so
// that each XCD walks a contiguous share of the (problem, block) list and
// neighbouring blocks share an L2.  A bijection on [0, total).
__device__ inline int xcd_order(int t, int total) {
  const int m = total >> 3, r = total & 7, x = t & 7, k = t >> 3;
  return x * m + (x < r ? x : r) + k;
}

__device__ inline int seg_find(const int* __restrict__ off, int n, int t) {
  int lo = 0, hi = n;   // off[lo] <= t < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- V-cycle kernels

// off[o][p + 1] = off[o][p] + (active[p] ? blocks[o][p] : 0), one thread per op.
__global__ void kb_plan(const int* __restrict__ blocks, int nops, int P, const int* __restrict__ active,
                        int* __restrict__ off) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nops) return;
  const int* bl = blocks + (size_t)o * P;
  int* of = off + (size_t)o * (P + 1);
  int acc = 0;
  of[0] = 0;
  for (int p = 0; p < P; ++p) {
    acc += active[p] ? bl[p] : 0;
    of[p + 1] = acc;
  }
}

template <typename T, int KIND>
__global__ void __launch_bounds__(256)
kb_level(const BLv<T>* __restrict__ lv, const int* __restrict__ ls, int P, int k, const int* __restrict__ off) {
  const int total = off[P];
  for (int tt = blockIdx.x; tt < total; tt += gridDim.x) {
    const int t = xcd_order(tt, total);
    const int p = seg_find(off, P, t);
    const int blk = t - off[p];
    const BLv<T>& e = lv[(size_t)(KIND == OP_FILL0 ? ls[p] - 1 : k) * P + p];
    if constexpr (KIND == OP_FILL0) {
      const int idx = blk * 256 + threadIdx.x;
      if (idx < 3 * e.L.N * e.L.N) e.w[idx] = T(0);
    } else if constexpr (KIND == OP_RES) {
      res_ib_body<T>(e.L, e.b, e.w, e.r, e.nres, blk, e.nibr);
    } else if constexpr (KIND == OP_RESID) {
      // residual before the restriction: Stokes part and elastic term in one
      // pass; the restriction subtracts the elastic term
      res_ib_body<T>(e.L, e.b, e.w, e.r, e.nres, blk, e.nibr);
    } else if constexpr (KIND == OP_RESTRICT) {
      restrict_body<T>(e.L.N, e.r, e.bc, e.wc, blk, e.L.yib);
    } else if constexpr (KIND == OP_PROLONG) {
      prolong_body<T>(e.L.N, e.wc, e.w, blk);
    }
  }
}

// from_zero: the first phase of a level's pre-smoothing, where the iterate
// is zero -- the boxes read b as the residual and no elastic term.
template <typename T>
__global__ void __launch_bounds__(64)
kb_box(const BLv<T>* __restrict__ lv, int P, int k, int colour, const int* __restrict__ off, int from_zero) {
  const int total = off[P];
  for (int tt = blockIdx.x; tt < total; tt += gridDim.x) {
    const int t = xcd_order(tt, total);
    const int p = seg_find(off, P, t);
    const BLv<T>& e = lv[(size_t)k * P + p];
    LevelView<T> L = e.L;
    if (from_zero) L.yib = nullptr;
    box_body<T>(L, from_zero ? e.b : e.r, e.w, colour, t - off[p]);
    __syncthreads();   // the box's LDS is reused by the next box of this workgroup
  }
}

// 8 x 8 boxes: tiles are (problem, box, row block), the four row blocks of a
// box adjacent (one XCD).
template <typename T>
__global__ void __launch_bounds__(kBigBoxLanes)
kb_box_big(const BLv<T>* __restrict__ lv, int P, int k, int colour, const int* __restrict__ off, int from_zero) {
  const int total = off[P];
  for (int tt = blockIdx.x; tt < total; tt += gridDim.x) {
    const int t = xcd_order(tt, total);
    const int p = seg_find(off, P, t);
    const BLv<T>& e = lv[(size_t)k * P + p];
    const int q = t - off[p];
    LevelView<T> L = e.L;
    if (from_zero) L.yib = nullptr;
    box_body_big<T>(L, from_zero ? e.b : e.r, e.w, colour, q / kBigBoxRowBlocks, q % kBigBoxRowBlocks);
    __syncthreads();   // the box's LDS is reused by the next tile of this workgroup
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) kb_tail(const TailArgs<T>* __restrict__ A, const int* __restrict__ active) {
  if (!active[blockIdx.x]) return;
  tail_body_n<T>(A[blockIdx.x]);
}

// ---------------------------------------------------------------- Krylov kernels (FP64)

// Residual of the outer operator: start ? V_0 = b - A x : V_{j+1} = A Z_j.
__global__ void __launch_bounds__(256) kb_resid0(BSet S, const BKry* __restrict__ K, int start) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const int j = S.j[s];
  const size_t n0 = q.n0;
  if (start) residual_body<double>(q.v0, q.b, q.x, q.V, blockIdx.x - S.off[s]);
  else residual_body<double>(q.v0, nullptr, q.Z + j * n0, q.V + (j + 1) * n0, blockIdx.x - S.off[s]);
}

__global__ void __launch_bounds__(256) kb_ibrows0(BSet S, const BKry* __restrict__ K, int start) {
  const int s = seg_find(S.off2, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const int j = S.j[s];
  const size_t n0 = q.n0;
  const int blk = blockIdx.x - S.off2[s];
  if (start) ib_rows_body<double>(q.v0, q.x, q.V, 2, blk % q.nibx, blk / q.nibx, q.nibx);
  else ib_rows_body<double>(q.v0, q.Z + j * n0, q.V + (j + 1) * n0, 1, blk % q.nibx, blk / q.nibx, q.nibx);
}

// Partial dot products, the per-problem partition of k_multidot (256
// workgroups striding over the vector).  kind 0: <V_0, V_0>; 1: <V_i, V_{j+1}>
// for i <= j; 2: <V_{j+1}, V_{j+1}>; 3: <b, b>.
#define BMD_GROUP 8
__global__ void __launch_bounds__(256) kb_multidot(BSet S, const BKry* __restrict__ K, int kind) {
  __shared__ double sh[BMD_GROUP][256];
  const int s = blockIdx.z;
  const BKry& q = K[S.p[s]];
  const int j = S.j[s];
  const size_t n = q.n0;
  const int nvec = kind == 1 ? j + 1 : 1;
  const int g0 = blockIdx.y * BMD_GROUP;
  if (g0 >= nvec) return;
  const int ng = min(BMD_GROUP, nvec - g0);
  const double* V;
  const double* w;
  size_t ldv = 0;
  if (kind == 0) { V = q.V; w = q.V; }
  else if (kind == 1) { V = q.V; w = q.V + (j + 1) * n; ldv = n; }
  else if (kind == 2) { V = q.V + (j + 1) * n; w = V; }
  else { V = q.b; w = q.b; }
  double acc[BMD_GROUP];
  // rows past the group's last vector repeat it (unconditional loads, as in
  // k_multidot; their sums are never stored)
  const double* Vc[BMD_GROUP];
#pragma unroll
  for (int c = 0; c < BMD_GROUP; ++c) {
    acc[c] = 0.0;
    Vc[c] = V + (size_t)(g0 + min(c, ng - 1)) * ldv;
  }
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)256 * 256) {
    const double we = w[e];
#pragma unroll
    for (int c = 0; c < BMD_GROUP; ++c) acc[c] += Vc[c][e] * we;
  }
#pragma unroll
  for (int c = 0; c < BMD_GROUP; ++c) sh[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int c = 0; c < BMD_GROUP; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < ng) q.partial[(size_t)(g0 + threadIdx.x) * 256 + blockIdx.x] = sh[threadIdx.x][0];
}

// Sum of the 256 partials of each dot (k_reduce's tree).  kind 0 -> scal[0];
// 1 -> column j of H; 3 -> hc (second Gram-Schmidt pass).
__global__ void __launch_bounds__(256) kb_reduce(BSet S, const BKry* __restrict__ K, int kind) {
  __shared__ double sh[256];
  const int s = blockIdx.y;
  const BKry& q = K[S.p[s]];
  const int j = S.j[s];
  const int nvec = kind == 0 ? 1 : j + 1;
  const int v = blockIdx.x;
  if (v >= nvec) return;
  double a = 0.0;
  for (int b = threadIdx.x; b < 256; b += 256) a += q.partial[(size_t)v * 256 + b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* out = kind == 0 ? q.scal : (kind == 1 ? q.H + (size_t)j * q.ldh : q.hc);
    out[v] = sh[0];
  }
}

// ||V_{j+1}||^2 into H(j+1, j) and scal[1] (k_reduce2).
__global__ void __launch_bounds__(256) kb_reduce2(BSet S, const BKry* __restrict__ K) {
  __shared__ double sh[256];
  const BKry& q = K[S.p[blockIdx.x]];
  const int j = S.j[blockIdx.x];
  double a = 0.0;
  for (int b = threadIdx.x; b < 256; b += 256) a += q.partial[b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    q.H[(size_t)j * q.ldh + j + 1] = sh[0];
    q.scal[1] = sh[0];
  }
}

// V_{j+1} -= sum_i c_i V_i (pass 1: c = H(:, j); pass 2: c = hc, added into H(:, j)).
__global__ void __launch_bounds__(256) kb_update_acc(BSet S, const BKry* __restrict__ K, int pass) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const int j = S.j[s], nvec = j + 1;
  const size_t n = q.n0;
  const int blk = blockIdx.x - S.off[s];
  double* col = q.H + (size_t)j * q.ldh;
  const double* coef = pass == 1 ? col : q.hc;
  double* acc = pass == 1 ? nullptr : col;
  const size_t e = (size_t)blk * 256 + threadIdx.x;
  if (acc && blk == 0)
    for (int t = threadIdx.x; t < nvec; t += blockDim.x) acc[t] += coef[t];
  if (e >= n) return;
  double sum = 0.0;
  // unrolled so that eight basis loads are in flight; the sum keeps its order
#pragma unroll 8
  for (int v = 0; v < nvec; ++v) sum += coef[v] * q.V[(size_t)v * n + e];
  q.V[(j + 1) * n + e] -= sum;
}

// V_{j+1} /= ||V_{j+1}||, and the Givens step of column j (k_scale_givens).
__global__ void __launch_bounds__(256) kb_scale_givens(BSet S, const BKry* __restrict__ K) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const int j = S.j[s];
  const size_t n = q.n0;
  const int blk = blockIdx.x - S.off[s];
  const size_t e = (size_t)blk * 256 + threadIdx.x;
  const double nrm = sqrt(q.scal[1]);
  double* w = q.V + (j + 1) * n;
  if (e < n) w[e] = nrm > 0.0 ? w[e] / nrm : 0.0;
  if (blk != 0 || threadIdx.x != 0) return;
  double* col = q.H + (size_t)j * q.ldh;
  col[j + 1] = nrm;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = q.cs[i] * a + q.sn[i] * b;
    col[i + 1] = -q.sn[i] * a + q.cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double d = hypot(a, b);
  q.cs[j] = a / d;
  q.sn[j] = b / d;
  col[j] = d;
  col[j + 1] = 0.0;
  q.g[j + 1] = -q.sn[j] * q.g[j];
  q.g[j] = q.cs[j] * q.g[j];
  const double est = fabs(q.g[j + 1]);
  q.flags[0] = est;
  q.flags[1] = (est <= q.target || nrm == 0.0) ? 1.0 : 0.0;
  q.flags[2] = (isfinite(est) && isfinite(d)) ? 0.0 : 1.0;
}

// Start of an Arnoldi cycle: V_0 /= ||V_0|| and g = beta e_1.
__global__ void __launch_bounds__(256) kb_start(BSet S, const BKry* __restrict__ K) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const size_t n = q.n0;
  const int blk = blockIdx.x - S.off[s];
  const size_t e = (size_t)blk * 256 + threadIdx.x;
  const double nrm = sqrt(q.scal[0]);
  if (e < n) q.V[e] = nrm > 0.0 ? q.V[e] / nrm : 0.0;
  if (blk == 0)
    for (int t = threadIdx.x; t < q.m + 2; t += blockDim.x) q.g[t] = t == 0 ? S.beta[s] : 0.0;
}

// y = R^{-1} g over the leading k x k block, one thread per problem.
__global__ void kb_backsolve(BSet S, const BKry* __restrict__ K) {
  if (threadIdx.x != 0) return;
  const BKry& q = K[S.p[blockIdx.x]];
  const int k = S.j[blockIdx.x];
  for (int i = k - 1; i >= 0; --i) {
    double sum = q.g[i];
    for (int c = i + 1; c < k; ++c) sum -= q.H[(size_t)c * q.ldh + i] * q.y[c];
    q.y[i] = sum / q.H[(size_t)i * q.ldh + i];
  }
}

// x += Z y over the k stored directions.
__global__ void __launch_bounds__(256) kb_update_x(BSet S, const BKry* __restrict__ K) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const int k = S.j[s];
  const size_t n = q.n0;
  const size_t e = (size_t)(blockIdx.x - S.off[s]) * 256 + threadIdx.x;
  if (e >= n) return;
  double sum = 0.0;
  // unrolled so that eight basis loads are in flight; the sum keeps its order
#pragma unroll 8
  for (int v = 0; v < k; ++v) sum += q.y[v] * q.Z[(size_t)v * n + e];
  q.x[e] += 1.0 * sum;
}

// V-cycle input b0 = V_j (in the V-cycle precision) and output Z_j = w0.
template <typename T>
__global__ void __launch_bounds__(256) kb_to_b0(BSet S, const BKry* __restrict__ K) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const size_t e = (size_t)(blockIdx.x - S.off[s]) * 256 + threadIdx.x;
  if (e < (size_t)q.n0) static_cast<T*>(q.b0)[e] = (T)q.V[(size_t)S.j[s] * q.n0 + e];
}
template <typename T>
__global__ void __launch_bounds__(256) kb_from_w0(BSet S, const BKry* __restrict__ K) {
  const int s = seg_find(S.off, S.n, blockIdx.x);
  const BKry& q = K[S.p[s]];
  const size_t e = (size_t)(blockIdx.x - S.off[s]) * 256 + threadIdx.x;
  if (e < (size_t)q.n0) q.Z[(size_t)S.j[s] * q.n0 + e] = (double)static_cast<const T*>(q.w0)[e];
}

// out[4p..4p+3] = scal[0], flags[0..2] of every problem.
__global__ void kb_gather(const BKry* __restrict__ K, int P, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  out[4 * p] = K[p].scal[0];
  out[4 * p + 1] = K[p].flags[0];
  out[4 * p + 2] = K[p].flags[1];
  out[4 * p + 3] = K[p].flags[2];
}

struct BOp {
  int kind, k, colour;
  int cap;
  int from_zero;   // box op of the first pre-smoothing phase (iterate zero, no residual op before it)
};

// Host-side slot set of a round, mirrored into the round buffer.
struct HostSet {
  std::vector<int> p, j, off, off2;
  std::vector<double> beta;
  void clear() { p.clear(); j.clear(); off.assign(1, 0); off2.assign(1, 0); beta.clear(); }
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct ibmg_batch {
  int P = 0, prec = IBMG_FP64, Kmax = 0;
  hipStream_t stream = nullptr, cap = nullptr;
  std::vector<hipStream_t> work;   // per-problem setup and step-end work, kWorkStreams-way concurrent
  std::vector<ibmg_handle*> h;
  std::vector<size_t> sub_off;
  size_t need = 0;
  char* ws = nullptr;
  // device tables (offsets into ws)
  size_t o_blv = 0, o_tail = 0, o_kry = 0, o_ls = 0, o_blocks = 0, o_off = 0, o_round = 0, o_gather = 0;
  size_t blv_bytes = 0, tail_bytes = 0, round_bytes = 0;
  std::vector<BOp> ops;
  std::vector<int> blocks;     // [op][P] workgroups of each op per problem
  std::vector<int> ls;         // first LDS-resident level per problem
  size_t tail_lds = 0;
  // host mirrors
  std::vector<char> blv_h, tail_h;
  std::vector<BKry> kry_h;
  char* round_h = nullptr;     // pinned
  double* gather_h = nullptr;  // pinned
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true, launch_error = false;
  int64_t rounds = 0;

  template <typename T> T* d(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Round buffer layout: active[P], then four slot sets (end, start, begin-cycle,
// inner), each p[P], j[P], off[P+1], off2[P+1], beta[P].
constexpr int kSets = 5;
enum { SET_END = 0, SET_START, SET_BEGIN, SET_INNER, SET_INNER32 };

size_t set_bytes(int P) { return (4 * (size_t)P + 2) * sizeof(int) + (size_t)P * sizeof(double) + 64; }
size_t round_bytes(int P) { return ((size_t)P * sizeof(int) + 255) / 256 * 256 + kSets * ((set_bytes(P) + 255) / 256 * 256); }

size_t set_base(int P, int set) {
  return ((size_t)P * sizeof(int) + 255) / 256 * 256 + (size_t)set * ((set_bytes(P) + 255) / 256 * 256);
}

// Write a host set into the pinned round image and return its device view.
BSet pack_set(ibmg_batch* B, int set, const HostSet& hs) {
  const int P = B->P;
  const size_t base = set_base(P, set);
  char* hb = B->round_h + base;
  char* db = B->ws + B->o_round + base;
  const int n = (int)hs.p.size();
  int* hp = reinterpret_cast<int*>(hb);
  int* hj = hp + P;
  int* hoff = hj + P;
  int* hoff2 = hoff + P + 1;
  double* hbeta = reinterpret_cast<double*>(((uintptr_t)(hoff2 + P + 1) + 7) & ~(uintptr_t)7);
  for (int i = 0; i < n; ++i) {
    hp[i] = hs.p[i];
    hj[i] = hs.j[i];
    hbeta[i] = hs.beta.empty() ? 0.0 : hs.beta[i];
  }
  for (int i = 0; i <= n; ++i) {
    hoff[i] = hs.off[i];
    hoff2[i] = hs.off2[i];
  }
  BSet S;
  S.n = n;
  S.p = reinterpret_cast<const int*>(db + ((char*)hp - hb));
  S.j = reinterpret_cast<const int*>(db + ((char*)hj - hb));
  S.off = reinterpret_cast<const int*>(db + ((char*)hoff - hb));
  S.off2 = reinterpret_cast<const int*>(db + ((char*)hoff2 - hb));
  S.beta = reinterpret_cast<const double*>(db + ((char*)hbeta - hb));
  return S;
}

// ---------------------------------------------------------------- schedule

template <typename T>
void launch_op(ibmg_batch* B, hipStream_t s, int o) {
  const BOp& op = B->ops[o];
  const BLv<T>* lv = B->d<BLv<T>>(B->o_blv);
  const int* ls = B->d<int>(B->o_ls);
  const int* off = B->d<int>(B->o_off) + (size_t)o * (B->P + 1);
  const int P = B->P;
  switch (op.kind) {
    case OP_FILL0: kb_level<T, OP_FILL0><<<op.cap, 256, 0, s>>>(lv, ls, P, 0, off); break;
    case OP_RES: kb_level<T, OP_RES><<<op.cap, 256, 0, s>>>(lv, ls, P, op.k, off); break;
    case OP_RESID: kb_level<T, OP_RESID><<<op.cap, 256, 0, s>>>(lv, ls, P, op.k, off); break;
    case OP_RESTRICT: kb_level<T, OP_RESTRICT><<<op.cap, 256, 0, s>>>(lv, ls, P, op.k, off); break;
    case OP_PROLONG: kb_level<T, OP_PROLONG><<<op.cap, 256, 0, s>>>(lv, ls, P, op.k, off); break;
    case OP_BOX: kb_box<T><<<op.cap, 64, 0, s>>>(lv, P, op.k, op.colour, off, op.from_zero); break;
    case OP_BOX8: kb_box_big<T><<<op.cap, kBigBoxLanes, 0, s>>>(lv, P, op.k, op.colour, off, op.from_zero); break;
  }
}

// The batched V-cycle on the fixed per-problem buffers b0 -> w0 of the
// problems marked active in the round buffer.
template <typename T>
void bvcycle(ibmg_batch* B, hipStream_t s) {
  const int nops = (int)B->ops.size();
  const int* active = B->d<int>(B->o_round);
  kb_plan<<<(nops + 63) / 64, 64, 0, s>>>(B->d<int>(B->o_blocks), nops, B->P, active, B->d<int>(B->o_off));
  // descent (FILL0, then per step k, largest grids first: pre-smoothing
  // phases, residual, elastic rows, restriction), the LDS-resident tail of
  // every problem, then the ascent (prolongation, post-smoothing)
  for (int o = 0; o < nops; ++o) {
    if (B->ops[o].kind == OP_TAIL)
      kb_tail<T><<<B->P, 1024, B->tail_lds, s>>>(B->d<TailArgs<T>>(B->o_tail), active);
    else
      launch_op<T>(B, s, o);
  }
}

// Build the op list and the workgroups each op needs per problem.
void build_schedule(ibmg_batch* B) {
  const int P = B->P;
  B->ls.assign(P, 0);
  B->Kmax = 0;
  int nu1 = 0, nu2 = 0, ncol = 0;
  for (int p = 0; p < P; ++p) {
    B->ls[p] = tail_start(B->h[p]);
    B->Kmax = std::max(B->Kmax, B->ls[p]);
    nu1 = std::max(nu1, B->h[p]->nu1);
    nu2 = std::max(nu2, B->h[p]->nu2);
    ncol = std::max(ncol, B->h[p]->ncol);
  }
  B->ops.clear();
  auto add = [&](int kind, int k, int colour, int sweep, int post, int from_zero = 0) {
    BOp op{kind, k, colour, 0, from_zero};
    int total = 0;
    for (int p = 0; p < P; ++p) {
      const ibmg_handle* hp = B->h[p];
      const int lsp = B->ls[p];
      int nb = 0;
      if (kind == OP_TAIL) {
        nb = 0;
      } else if (kind == OP_FILL0) {
        nb = lsp > 0 ? (int)nblk(hp->n0()) : 0;
      } else if (k < lsp) {
        const int l = lsp - 1 - k;
        const LevelBufs& L = hp->L[l];
        const size_t NN = (size_t)L.N * L.N;
        const bool ib = hp->M > 0 && hp->K != 0.0;
        const bool in_sweep = sweep < (post ? hp->nu2 : hp->nu1) && colour < hp->ncol_l[l];
        switch (kind) {
          case OP_RES:
            nb = in_sweep ? (int)nblk(3 * NN) + (ib ? 2 * ib_blocks(L.maxact) : 0) : 0;
            break;
          case OP_BOX: nb = in_sweep && hp->n <= 4 ? colour_count(hp->ncol_l[l], L.nb) : 0; break;
          case OP_BOX8: nb = in_sweep && hp->n == 8 ? colour_count(hp->ncol_l[l], L.nb) * kBigBoxRowBlocks : 0; break;
          case OP_RESID: nb = (int)nblk(3 * NN) + (ib ? 2 * ib_blocks(L.maxact) : 0); break;
          case OP_RESTRICT: nb = (int)nblk(3 * NN / 4); break;
          case OP_PROLONG: nb = (int)nblk(3 * NN); break;
        }
      }
      B->blocks.push_back(nb);
      total += nb;
    }
    op.cap = std::max(1, std::min(total, kind == OP_BOX ? kCapBox : kind == OP_BOX8 ? kCapBox8 : kCap256));
    B->ops.push_back(op);
  };
  B->blocks.clear();
  add(OP_FILL0, 0, 0, 0, 0);
  for (int k = B->Kmax - 1; k >= 0; --k) {
    for (int q = 0; q < nu1; ++q)
      for (int c = 0; c < ncol; ++c) {
        // the level's iterate is zero before its first phase (FILL0 or the
        // restriction into it cleared it): no residual op, boxes read b
        const int fz = q == 0 && c == 0;
        if (!fz) add(OP_RES, k, c, q, 0);
        add(OP_BOX, k, c, q, 0, fz);
        add(OP_BOX8, k, c, q, 0, fz);
      }
    add(OP_RESID, k, 0, 0, 0);
    add(OP_RESTRICT, k, 0, 0, 0);
  }
  add(OP_TAIL, 0, 0, 0, 0);   // the LDS-resident tail of every problem
  for (int k = 0; k < B->Kmax; ++k) {
    add(OP_PROLONG, k, 0, 0, 1);
    for (int q = 0; q < nu2; ++q)
      for (int c = 0; c < ncol; ++c) {
        add(OP_RES, k, c, q, 1);
        add(OP_BOX, k, c, q, 1);
        add(OP_BOX8, k, c, q, 1);
      }
  }
  // drop ops no problem takes part in (the tail marker stays)
  std::vector<BOp> ops;
  std::vector<int> blocks;
  for (size_t o = 0; o < B->ops.size(); ++o) {
    int total = 0;
    for (int p = 0; p < P; ++p) total += B->blocks[o * P + p];
    if (total == 0 && B->ops[o].kind != OP_TAIL) continue;
    ops.push_back(B->ops[o]);
    blocks.insert(blocks.end(), B->blocks.begin() + o * P, B->blocks.begin() + (o + 1) * P);
  }
  B->ops.swap(ops);
  B->blocks.swap(blocks);
}

// Per-step device tables: level views (rho/dt changes with dt), tail
// arguments and Krylov state of every problem.
template <typename T>
void fill_tables(ibmg_batch* B) {
  const int P = B->P;
  B->blv_h.assign(sizeof(BLv<T>) * std::max(1, B->Kmax) * P, 0);
  B->tail_h.assign(sizeof(TailArgs<T>) * P, 0);
  BLv<T>* lv = reinterpret_cast<BLv<T>*>(B->blv_h.data());
  TailArgs<T>* ta = reinterpret_cast<TailArgs<T>*>(B->tail_h.data());
  for (int p = 0; p < P; ++p) {
    ibmg_handle* h = B->h[p];
    const bool ib = h->has_ib;
    T* b0 = h->prec == IBMG_FP32 ? reinterpret_cast<T*>(h->p<float>(h->b0f)) : reinterpret_cast<T*>(h->p<double>(h->b0g));
    T* w0 = h->prec == IBMG_FP32 ? reinterpret_cast<T*>(h->p<float>(h->w0f)) : reinterpret_cast<T*>(h->p<double>(h->w0g));
    const int lsp = B->ls[p];
    LevelView<T> v[IBMG_MAX_LEVELS];
    for (int l = 0; l < h->levels; ++l) {
      v[l] = view<T>(h, l);
      if (!ib) v[l].ib_index = nullptr;
    }
    for (int k = 0; k < lsp; ++k) {
      const int l = lsp - 1 - k;
      BLv<T>& e = lv[(size_t)k * P + p];
      e.L = v[l];
      e.b = l == 0 ? b0 : h->p<T>(h->L[l].b);
      e.w = l == 0 ? w0 : h->p<T>(h->L[l].w);
      e.r = h->p<T>(h->L[l].r);
      e.bc = h->p<T>(h->L[l + 1].b);
      e.wc = h->p<T>(h->L[l + 1].w);
      const size_t NN = (size_t)v[l].N * v[l].N;
      e.nres = (int)nblk(3 * NN);
      e.nibr = 2 * ib_blocks(v[l].maxact);
    }
    TailArgs<T>& A = ta[p];
    for (int l = 0; l < h->levels; ++l) A.v[l] = v[l];
    A.ls = lsp; A.L = h->levels; A.nu1 = h->nu1; A.nu2 = h->nu2; A.ib = ib ? 1 : 0; A.nr = h->nr;
    A.b_in = lsp == 0 ? b0 : h->p<T>(h->L[lsp].b);
    A.w_out = lsp == 0 ? w0 : h->p<T>(h->L[lsp].w);
    A.cainv = h->p<double>(h->cainv);
    BKry& q = B->kry_h[p];
    q.v0 = view<double>(h, 0);
    q.b = h->p<double>(h->bvec);
    q.x = h->p<double>(h->xvec);
    q.V = h->p<double>(h->V); q.Z = h->p<double>(h->Z); q.H = h->p<double>(h->H); q.g = h->p<double>(h->g);
    q.cs = h->p<double>(h->cs); q.sn = h->p<double>(h->sn); q.y = h->p<double>(h->y);
    q.flags = h->p<double>(h->flags); q.scal = h->p<double>(h->scal); q.hc = h->p<double>(h->hc);
    q.partial = h->p<double>(h->partial);
    q.b0 = b0; q.w0 = w0;
    q.n0 = (long long)h->n0();
    q.ldh = h->mb + 1; q.m = h->mb;
    q.nibx = ib_blocks(h->L[0].maxact);
    q.target = 0.0;   // set by the solve once ||b|| is known
  }
}

int upload_tables(ibmg_batch* B) {
  hipStream_t s = B->stream;
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_blv, B->blv_h.data(), B->blv_h.size(), hipMemcpyHostToDevice, s));
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_tail, B->tail_h.data(), B->tail_h.size(), hipMemcpyHostToDevice, s));
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_kry, B->kry_h.data(), B->kry_h.size() * sizeof(BKry), hipMemcpyHostToDevice,
                          s));
  IBMG_HIP(hipStreamSynchronize(s));
  return IBMG_OK;
}

int capture(ibmg_batch* B) {
  std::lock_guard<std::mutex> capture_lock(capture_mutex());
  IBMG_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  if (B->prec == IBMG_FP32) bvcycle<float>(B, B->cap);
  else bvcycle<double>(B, B->cap);
  const hipError_t e = hipStreamEndCapture(B->cap, &B->graph);
  if (e != hipSuccess) return IBMG_EHIP;
  IBMG_HIP(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
  return IBMG_OK;
}

// Workgroup prefix of a slot set: element blocks and elastic-row blocks.
void add_slot(ibmg_batch* B, HostSet& hs, int p, int j, double beta = 0.0) {
  const ibmg_handle* h = B->h[p];
  hs.p.push_back(p);
  hs.j.push_back(j);
  hs.beta.push_back(beta);
  hs.off.push_back(hs.off.back() + (int)nblk(h->n0()));
  hs.off2.push_back(hs.off2.back() + (h->has_ib ? 2 * ib_blocks(h->L[0].maxact) : 0));
}

// ---------------------------------------------------------------- lockstep FGMRES

enum { ST_START = 0, ST_INNER, ST_DONE };

struct PState {
  int state = ST_START, j = 0, total = 0, k_end = -1, rc = IBMG_OK;
  bool begin = false;
  bool fb64 = false;          // FP32 V-cycle stalled: this solve goes on with the FP64 one
  std::vector<double> hist;   // Arnoldi estimate after each iteration
  double bnorm = 0, beta = 0, est = INFINITY, target = 0;
  double best = INFINITY;     // smallest true residual of the solve so far (iterate kept in xbest)
  ibmg_stats st{};
};

int batch_solve(ibmg_batch* B, std::vector<PState>& ps) {
  const int P = B->P;
  hipStream_t s = B->stream;
  const BKry* K = B->d<BKry>(B->o_kry);
  double* gat = B->d<double>(B->o_gather);
  // ||b|| of every problem
  HostSet all;
  all.clear();
  for (int p = 0; p < P; ++p) add_slot(B, all, p, 0);
  BSet S0 = pack_set(B, SET_START, all);
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_round, B->round_h, B->round_bytes, hipMemcpyHostToDevice, s));
  kb_multidot<<<dim3(256, 1, P), 256, 0, s>>>(S0, K, 3);
  kb_reduce<<<dim3(1, P), 256, 0, s>>>(S0, K, 0);
  kb_gather<<<(P + 63) / 64, 64, 0, s>>>(K, P, gat);
  IBMG_HIP(hipMemcpyAsync(B->gather_h, gat, 4 * (size_t)P * sizeof(double), hipMemcpyDeviceToHost, s));
  IBMG_HIP(hipStreamSynchronize(s));
  bool any_target = false;
  for (int p = 0; p < P; ++p) {
    PState& q = ps[p];
    q.bnorm = std::sqrt(B->gather_h[4 * p]);
    q.st.bnorm = q.bnorm;
    if (!std::isfinite(q.bnorm)) { q.rc = IBMG_ENONFINITE; q.state = ST_DONE; continue; }
    if (q.bnorm == 0.0) {
      const size_t n0 = B->h[p]->n0();
      k_fill<double><<<nblk(n0), 256, 0, s>>>(B->h[p]->p<double>(B->h[p]->xvec), n0, 0.0);
      q.st.converged = 1;
      q.state = ST_DONE;
      continue;
    }
    q.target = B->h[p]->rtol * q.bnorm;
    if (B->kry_h[p].target != q.target) { B->kry_h[p].target = q.target; any_target = true; }
  }
  if (any_target)
    IBMG_HIP(hipMemcpyAsync(B->ws + B->o_kry, B->kry_h.data(), P * sizeof(BKry), hipMemcpyHostToDevice, s));
  HostSet E, S, G, I, I32;
  int* active_h = reinterpret_cast<int*>(B->round_h);
  for (;;) {
    E.clear(); S.clear(); G.clear(); I.clear(); I32.clear();
    for (int p = 0; p < P; ++p) {
      PState& q = ps[p];
      if (q.state == ST_DONE) continue;
      if (q.state == ST_START) {
        if (q.k_end >= 0) add_slot(B, E, p, q.k_end);
        add_slot(B, S, p, 0);
      } else {
        if (q.begin) add_slot(B, G, p, 0, q.beta);
        add_slot(B, I, p, q.j);
        if (!q.fb64) add_slot(B, I32, p, q.j);
      }
    }
    if (S.p.empty() && I.p.empty()) break;
    for (int p = 0; p < P; ++p) active_h[p] = 0;
    for (int p : I32.p) active_h[p] = 1;
    const BSet sE = pack_set(B, SET_END, E), sS = pack_set(B, SET_START, S), sG = pack_set(B, SET_BEGIN, G),
               sI = pack_set(B, SET_INNER, I), sI32 = pack_set(B, SET_INNER32, I32);
    IBMG_HIP(hipMemcpyAsync(B->ws + B->o_round, B->round_h, B->round_bytes, hipMemcpyHostToDevice, s));
    if (sE.n) {
      kb_backsolve<<<sE.n, 64, 0, s>>>(sE, K);
      kb_update_x<<<E.off.back(), 256, 0, s>>>(sE, K);
    }
    if (sS.n) {
      kb_resid0<<<S.off.back(), 256, 0, s>>>(sS, K, 1);
      if (S.off2.back() > 0) kb_ibrows0<<<S.off2.back(), 256, 0, s>>>(sS, K, 1);
      kb_multidot<<<dim3(256, 1, sS.n), 256, 0, s>>>(sS, K, 0);
      kb_reduce<<<dim3(1, sS.n), 256, 0, s>>>(sS, K, 0);
    }
    if (sG.n) kb_start<<<G.off.back(), 256, 0, s>>>(sG, K);
    if (sI.n) {
      int jmax = 0;
      for (int j : I.j) jmax = std::max(jmax, j);
      const int groups = (jmax + 1 + BMD_GROUP - 1) / BMD_GROUP;
      const int ne = I.off.back(), ne32 = I32.off.back();
      if (sI32.n) {
        if (B->prec == IBMG_FP32) kb_to_b0<float><<<ne32, 256, 0, s>>>(sI32, K);
        else kb_to_b0<double><<<ne32, 256, 0, s>>>(sI32, K);
        if (B->use_graph) {
          if (!B->gexec) {
            const int rc = capture(B);
            if (rc) return rc;
          }
          IBMG_HIP(hipGraphLaunch(B->gexec, s));
        } else if (B->prec == IBMG_FP32) {
          bvcycle<float>(B, s);
        } else {
          bvcycle<double>(B, s);
        }
        if (B->prec == IBMG_FP32) kb_from_w0<float><<<ne32, 256, 0, s>>>(sI32, K);
        else kb_from_w0<double><<<ne32, 256, 0, s>>>(sI32, K);
      }
      // problems whose FP32 V-cycle stalled: their own FP64 V-cycle
      for (size_t q = 0; q < I.p.size(); ++q) {
        const int p = I.p[q];
        if (!ps[p].fb64) continue;
        ibmg_handle* hp = B->h[p];
        const size_t n0 = hp->n0();
        vcycle_fp64(hp, hp->p<double>(hp->V) + (size_t)I.j[q] * n0, hp->p<double>(hp->Z) + (size_t)I.j[q] * n0);
      }
      kb_resid0<<<ne, 256, 0, s>>>(sI, K, 0);
      if (I.off2.back() > 0) kb_ibrows0<<<I.off2.back(), 256, 0, s>>>(sI, K, 0);
      // classical Gram-Schmidt, twice; then H(j+1, j) and the Givens step
      kb_multidot<<<dim3(256, groups, sI.n), 256, 0, s>>>(sI, K, 1);
      kb_reduce<<<dim3(jmax + 1, sI.n), 256, 0, s>>>(sI, K, 1);
      kb_update_acc<<<ne, 256, 0, s>>>(sI, K, 1);
      kb_multidot<<<dim3(256, groups, sI.n), 256, 0, s>>>(sI, K, 1);
      kb_reduce<<<dim3(jmax + 1, sI.n), 256, 0, s>>>(sI, K, 3);
      kb_update_acc<<<ne, 256, 0, s>>>(sI, K, 2);
      kb_multidot<<<dim3(256, 1, sI.n), 256, 0, s>>>(sI, K, 2);
      kb_reduce2<<<sI.n, 256, 0, s>>>(sI, K);
      kb_scale_givens<<<ne, 256, 0, s>>>(sI, K);
    }
    kb_gather<<<(P + 63) / 64, 64, 0, s>>>(K, P, gat);
    IBMG_HIP(hipGetLastError());
    IBMG_HIP(hipMemcpyAsync(B->gather_h, gat, 4 * (size_t)P * sizeof(double), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    ++B->rounds;
    // same restart and best-iterate rules as the single-problem solve
    for (int p : S.p) {
      PState& q = ps[p];
      ibmg_handle* hp = B->h[p];
      const int m = hp->maxit;   // iteration cap over all cycles
      const size_t xb = hp->n0() * sizeof(double);
      q.k_end = -1;
      const double beta = std::sqrt(B->gather_h[4 * p]);
      if (!std::isfinite(beta)) { q.rc = IBMG_ENONFINITE; q.state = ST_DONE; continue; }
      q.st.rel_resid_true = beta / q.bnorm;
      if (beta <= q.target) { q.st.converged = 1; q.state = ST_DONE; continue; }
      if (beta < q.best) {
        q.best = beta;
        if (q.total < m)
          IBMG_HIP(hipMemcpyAsync(hp->p<double>(hp->xbest), hp->p<double>(hp->xvec), xb, hipMemcpyDeviceToDevice, s));
      }
      if (q.total >= m) {
        if (beta > q.best) {        // give back the best iterate
          IBMG_HIP(hipMemcpyAsync(hp->p<double>(hp->xvec), hp->p<double>(hp->xbest), xb, hipMemcpyDeviceToDevice,
                                  s));
          q.st.rel_resid_true = q.best / q.bnorm;
        }
        q.state = ST_DONE;
        continue;
      }
      q.beta = beta;
      q.begin = true;
      q.j = 0;
      q.state = ST_INNER;
    }
    for (int p : I.p) {
      PState& q = ps[p];
      const int m = B->h[p]->mb, cap = B->h[p]->maxit;
      q.begin = false;
      ++q.total;
      const double* f = B->gather_h + 4 * p + 1;
      q.est = f[0] / q.bnorm;
      if (f[2] != 0.0) { q.rc = IBMG_ENONFINITE; q.state = ST_DONE; continue; }
      q.hist.push_back(q.est);
      const int nh = (int)q.hist.size();
      if (B->prec == IBMG_FP32 && !q.fb64 && nh > kFallbackWindow && q.est > 0.9 * q.hist[nh - 1 - kFallbackWindow]) {
        q.fb64 = true;   // same stall test as the single-problem solve: restart with the FP64 V-cycle
        q.st.fallback = 1;
        q.k_end = q.j + 1;
        q.state = ST_START;
        continue;
      }
      if (f[1] != 0.0 || q.j + 1 >= m || q.total >= cap) {
        q.k_end = q.j + 1;
        q.state = ST_START;
      } else {
        ++q.j;
      }
    }
  }
  for (int p = 0; p < P; ++p) {
    PState& q = ps[p];
    q.st.iters = q.total;
    q.st.rel_resid_est = std::isfinite(q.est) ? q.est : q.st.rel_resid_true;
  }
  return IBMG_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int ibmg_batch_create(ibmg_batch** out, int32_t nprob, const ibmg_problem* probs, const ibmg_opts* opts,
                      void* stream) {
  if (!out || !probs || !opts || nprob < 1 || nprob > 4096) return IBMG_EINVAL;
  *out = nullptr;
  ibmg_batch* B = new (std::nothrow) ibmg_batch();
  if (!B) return IBMG_EINVAL;
  B->P = nprob;
  B->stream = (hipStream_t)stream;
  B->prec = opts[0].vcycle_prec;
  for (int p = 0; p < nprob; ++p) {
    ibmg_handle* h = nullptr;
    int rc = (opts[p].vcycle_prec != B->prec || opts[p].orth != IBMG_ORTH_CGS2 || probs[p].domain != IBMG_PERIODIC)
                 ? IBMG_EINVAL
                 : ibmg_create(&h, &probs[p], &opts[p], stream);
    if (rc) {
      for (ibmg_handle* q : B->h) ibmg_destroy(q);
      delete B;
      return rc;
    }
    B->h.push_back(h);
  }
  build_schedule(B);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    cur = (cur + 255) & ~(size_t)255;
    const size_t o = cur;
    cur += bytes;
    return o;
  };
  for (int p = 0; p < nprob; ++p) B->sub_off.push_back(take(B->h[p]->need));
  const size_t es = B->prec == IBMG_FP32 ? sizeof(float) : sizeof(double);
  const size_t blv = B->prec == IBMG_FP32 ? sizeof(BLv<float>) : sizeof(BLv<double>);
  const size_t tai = B->prec == IBMG_FP32 ? sizeof(TailArgs<float>) : sizeof(TailArgs<double>);
  B->o_blv = take(blv * std::max(1, B->Kmax) * nprob);
  B->o_tail = take(tai * nprob);
  B->o_kry = take(sizeof(BKry) * nprob);
  B->o_ls = take(sizeof(int) * nprob);
  B->o_blocks = take(sizeof(int) * B->blocks.size());
  B->o_off = take(sizeof(int) * B->ops.size() * (nprob + 1));
  B->round_bytes = round_bytes(nprob);
  B->o_round = take(B->round_bytes);
  B->o_gather = take(4 * sizeof(double) * nprob);
  B->need = cur + 256;
  B->kry_h.assign(nprob, BKry{});
  for (int p = 0; p < nprob; ++p) B->tail_lds = std::max(B->tail_lds, tail_lds(B->h[p], es));
  *out = B;
  return IBMG_OK;
}

int ibmg_batch_workspace_bytes(const ibmg_batch* B, size_t* bytes) {
  if (!B || !bytes) return IBMG_EINVAL;
  *bytes = B->need;
  return IBMG_OK;
}

int ibmg_batch_bind_workspace(ibmg_batch* B, void* dev, size_t bytes) {
  if (!B || !dev) return IBMG_EINVAL;
  char* base = (char*)(((uintptr_t)dev + 255) & ~(uintptr_t)255);
  if (bytes < B->need || (size_t)(base - (char*)dev) + B->need - 256 > bytes) return IBMG_ENOMEM;
  if (B->gexec) { (void)hipGraphExecDestroy(B->gexec); B->gexec = nullptr; }
  if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
  B->ws = base;
  for (int p = 0; p < B->P; ++p) {
    const int rc = bind(B->h[p], base + B->sub_off[p], B->h[p]->need, false);
    if (rc) return rc;
  }
  if (B->tail_lds > 65536) {
    const void* f = B->prec == IBMG_FP32 ? (const void*)kb_tail<float> : (const void*)kb_tail<double>;
    IBMG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)B->tail_lds));
  }
  if (!B->cap) IBMG_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  while ((int)B->work.size() < kWorkStreams) {
    hipStream_t w = nullptr;
    IBMG_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
    B->work.push_back(w);
  }
  if (!B->round_h) IBMG_HIP(hipHostMalloc((void**)&B->round_h, B->round_bytes, hipHostMallocDefault));
  if (!B->gather_h) IBMG_HIP(hipHostMalloc((void**)&B->gather_h, 4 * sizeof(double) * B->P, hipHostMallocDefault));
  std::memset(B->round_h, 0, B->round_bytes);
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_ls, B->ls.data(), sizeof(int) * B->P, hipMemcpyHostToDevice, B->stream));
  IBMG_HIP(hipMemcpyAsync(B->ws + B->o_blocks, B->blocks.data(), sizeof(int) * B->blocks.size(),
                          hipMemcpyHostToDevice, B->stream));
  IBMG_HIP(hipStreamSynchronize(B->stream));
  return IBMG_OK;
}

int ibmg_batch_set_graph(ibmg_batch* B, int on) {
  if (!B) return IBMG_EINVAL;
  B->use_graph = on != 0;
  return IBMG_OK;
}

int ibmg_batch_step(ibmg_batch* B, const double* dt, double* const* u, double* const* v, double* const* p,
                    double* const* X, const double* const* g_u, const double* const* g_v, ibmg_stats* out) {
  if (!B || !B->ws) return IBMG_ENOMEM;
  if (!dt || !u || !v || !p || !X) return IBMG_EINVAL;
  const int P = B->P;
  for (int q = 0; q < P; ++q) {
    if (!u[q] || !v[q] || !p[q] || (B->h[q]->M > 0 && !X[q])) return IBMG_EINVAL;
    if (!(dt[q] > 0.0) || !std::isfinite(dt[q])) return IBMG_EINVAL;
  }
  const double t0 = now_ms();
  hipStream_t s = B->stream;
  int rc;
  // the problems' setups and right-hand sides are independent: they run on
  // the work streams, round-robin, after the caller's stream has produced the
  // inputs; the solve runs on the handle's stream once they are all done
  IBMG_HIP(hipStreamSynchronize(s));
  auto on_work = [&](bool w) {
    for (int q = 0; q < P; ++q) B->h[q]->stream = w ? B->work[q % B->work.size()] : s;
  };
  auto sync_work = [&]() -> int {
    for (hipStream_t w : B->work) IBMG_HIP(hipStreamSynchronize(w));
    return IBMG_OK;
  };
  on_work(true);
  for (int q = 0; q < P; ++q)
    if ((rc = setup_launch(B->h[q], dt[q], X[q]))) { on_work(false); return rc; }
  if ((rc = sync_work())) { on_work(false); return rc; }
  for (int q = 0; q < P; ++q)
    if ((rc = setup_finish(B->h[q]))) { on_work(false); return rc; }
  for (int q = 0; q < P; ++q) {
    const double* gu = g_u ? g_u[q] : nullptr;
    const double* gv = g_v ? g_v[q] : nullptr;
    if ((rc = step_begin(B->h[q], dt[q], u[q], v[q], p[q], gu, gv))) { on_work(false); return rc; }
  }
  rc = sync_work();
  on_work(false);
  if (rc) return rc;
  if (B->prec == IBMG_FP32) fill_tables<float>(B);
  else fill_tables<double>(B);
  if ((rc = upload_tables(B))) return rc;
  for (int q = 0; q < P; ++q) B->h[q]->setup_ok = true;
  const double t1 = now_ms();
  std::vector<PState> ps(P);
  rc = batch_solve(B, ps);
  const double t2 = now_ms();
  if (rc < 0) return rc;
  int worst = IBMG_OK;
  for (int q = 0; q < P; ++q) {
    if (ps[q].rc < 0) return ps[q].rc;
    if (!ps[q].st.converged) worst = IBMG_NOT_CONVERGED;
  }
  IBMG_HIP(hipStreamSynchronize(s));
  on_work(true);
  for (int q = 0; q < P; ++q)
    if ((rc = step_end(B->h[q], dt[q], u[q], v[q], p[q], X[q]))) { on_work(false); return rc; }
  rc = sync_work();
  on_work(false);
  if (rc) return rc;
  const double t3 = now_ms();
  for (int q = 0; q < P; ++q) {
    B->h[q]->setup_ok = false;
    if (out) {
      out[q] = ps[q].st;
      out[q].t_setup_ms = t1 - t0;
      out[q].t_solve_ms = t2 - t1;
      out[q].t_step_ms = t3 - t0;
    }
  }
  return worst;
}

int ibmg_batch_rounds(const ibmg_batch* B, int64_t* rounds) {
  if (!B || !rounds) return IBMG_EINVAL;
  *rounds = B->rounds;
  return IBMG_OK;
}

int ibmg_batch_destroy(ibmg_batch* B) {
  if (!B) return IBMG_EINVAL;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  for (hipStream_t w : B->work) (void)hipStreamDestroy(w);
  if (B->round_h) (void)hipHostFree(B->round_h);
  if (B->gather_h) (void)hipHostFree(B->gather_h);
  for (ibmg_handle* h : B->h) ibmg_destroy(h);
  delete B;
  return IBMG_OK;
}

}  // extern "C"
