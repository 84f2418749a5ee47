// Per-step operator setup on gfx950: fibre forces, delta weights, point-to-box
// binning, the elasticity operator on every level as per-face coefficient
// windows, and the dense box factors.
//
// Paper references: fibre force and regularised delta (Sec. 2.2); lagged
// spreading/interpolation and the elimination M_0 = -dt K S L S^* (Sec. 2.3.2);
// Galerkin coarsening M_{l+1} = R M_l P with the Sec. 3.1 transfers
// (Sec. 3.2); box relaxation blocks (Sec. 5-6); plain boxes share one factor
// while boxes near the structure get their own, re-formed every step (Sec. 8).
#include <climits>
#include "common.h"
#include "gj.h"
#include "gj_reg.h"
#include "kernels.h"

// ---------------------------------------------------------------- a1: G = K L X
__global__ void __launch_bounds__(256)
k_fiber_force(int M, const int* __restrict__ prev, const int* __restrict__ next, double K,
              const double* __restrict__ X, double* __restrict__ G) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const int a = prev[k], b = next[k];
  G[2 * k] = K * (X[2 * a] - 2.0 * X[2 * k] + X[2 * b]);
  G[2 * k + 1] = K * (X[2 * a + 1] - 2.0 * X[2 * k + 1] + X[2 * b + 1]);
}

// ---------------------------------------------------------------- a3: finest patches
// Component 0 (u faces at (i, j + 1/2)) and 1 (v faces at (i + 1/2, j)), grid
// units.  The 4 x 4 patch starts at floor(s) - 1 in each direction, which
// contains the whole support |r| < 2 of either kernel.
__global__ void __launch_bounds__(256)
k_weights0(int M, int N, int kind, const double* __restrict__ X, int* __restrict__ org,
           double* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * M) return;
  const int comp = t / M, k = t % M;
  double sx = X[2 * k] * N, sy = X[2 * k + 1] * N;
  if (comp == 0) sy -= 0.5; else sx -= 0.5;
  const double fx = floor(sx), fy = floor(sy);
  const int i0 = (int)fx - 1, j0 = (int)fy - 1;
  double wx[4], wy[4];
  for (int a = 0; a < 4; ++a) {
    wx[a] = phi_kernel((double)(i0 + a) - sx, kind);
    wy[a] = phi_kernel((double)(j0 + a) - sy, kind);
  }
  double* o = w + (size_t)t * IBMG_PATCH;
  for (int b = 0; b < 4; ++b)
    for (int a = 0; a < 4; ++a) o[b * 4 + a] = wx[a] * wy[b];
  org[2 * t] = ((i0 % N) + N) % N;
  org[2 * t + 1] = ((j0 % N) + N) % N;
}

// ---------------------------------------------------------------- a2: point-to-box binning (finest)
__device__ inline void add_unique(int* a, int& n, int v) {
  for (int q = 0; q < n; ++q)
    if (a[q] == v) return;
  a[n++] = v;
}

// Boxes whose unknowns of component comp meet the 4 x 4 patch at (oi, oj).
// A u face on a box's left edge also belongs to the box on its left (shared
// edge unknowns are updated by both boxes, Sec. 6); likewise v in y.
__device__ inline void patch_boxes(int comp, int oi, int oj, int n, int N, int nb, int* ids, int& cnt) {
  int bxs[8], bys[8], nbx = 0, nby = 0;
  for (int a = 0; a < 4; ++a) {
    const int x = wrapi(oi + a, N), y = wrapi(oj + a, N);
    add_unique(bxs, nbx, x / n);
    if (comp == 0 && x % n == 0) add_unique(bxs, nbx, (x / n - 1 + nb) % nb);
    add_unique(bys, nby, y / n);
    if (comp == 1 && y % n == 0) add_unique(bys, nby, (y / n - 1 + nb) % nb);
  }
  for (int p = 0; p < nby; ++p)
    for (int q = 0; q < nbx; ++q) add_unique(ids, cnt, bys[p] * nb + bxs[q]);
}

__device__ inline int point_boxes(int k, int M, const int* org, int n, int N, int nb, int* ids) {
  int cnt = 0;
  for (int comp = 0; comp < 2; ++comp)
    patch_boxes(comp, org[(comp * M + k) * 2], org[(comp * M + k) * 2 + 1], n, N, nb, ids, cnt);
  return cnt;
}

__global__ void __launch_bounds__(256)
k_box_count(int M, const int* __restrict__ org, int n, int N, int nb, int* __restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  int ids[64];
  const int c = point_boxes(k, M, org, n, N, nb, ids);
  for (int q = 0; q < c; ++q) atomicAdd(&cnt[ids[q]], 1);
}

__global__ void __launch_bounds__(256)
k_box_fill(int M, const int* __restrict__ org, int n, int N, int nb, const int* __restrict__ start,
           int* __restrict__ cursor, int* __restrict__ list, int max_list) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  int ids[64];
  const int c = point_boxes(k, M, org, n, N, nb, ids);
  for (int q = 0; q < c; ++q) {
    const int pos = atomicAdd(&cursor[ids[q]], 1);
    const int at = start[ids[q]] + pos;
    if (at < max_list) list[at] = k;
  }
}

// Ascending point ids within each box (fixed summation order downstream).
// One workgroup per box: the box's list is staged in LDS and sorted there.
// Short lists (at most one entry per lane) place every entry at its rank (the
// number of smaller ids; ids in a box are distinct); longer ones, where points
// crowd into a box, run a bitonic network over the list padded to a power of
// two.  A list longer than the staging area is sorted in place by insertion,
// one lane (not met on the benchmark workloads).
constexpr int kSortCap = 4096, kSortLanes = 256;

__global__ void __launch_bounds__(kSortLanes)
k_box_sort(int nbox, const int* __restrict__ start, int* __restrict__ list, int max_list) {
  __shared__ int st[kSortCap];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= nbox) return;
  const int s = start[b], e = min(start[b + 1], max_list), m = e - s;
  if (m <= 1) return;
  if (m > kSortCap) {
    if (tid == 0)
      for (int i = s + 1; i < e; ++i) {
        const int v = list[i];
        int j = i - 1;
        while (j >= s && list[j] > v) { list[j + 1] = list[j]; --j; }
        list[j + 1] = v;
      }
    return;
  }
  if (m <= kSortLanes) {
    const int v = tid < m ? list[s + tid] : 0;
    if (tid < m) st[tid] = v;
    __syncthreads();
    if (tid < m) {
      int rank = 0;
      for (int q = 0; q < m; ++q) rank += st[q] < v;
      list[s + rank] = v;
    }
    return;
  }
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = tid; i < P; i += kSortLanes) st[i] = i < m ? list[s + i] : INT_MAX;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += kSortLanes) {
        const int l = i ^ j;
        if (l > i) {
          const int a = st[i], c = st[l];
          const bool up = (i & k) == 0;
          if ((a > c) == up) { st[i] = c; st[l] = a; }
        }
      }
      __syncthreads();
    }
  for (int i = tid; i < m; i += kSortLanes) list[s + i] = st[i];
}

// ---------------------------------------------------------------- multi-block exclusive scan
// Pass 1: each workgroup scans 1024 entries (4 per thread), writes the local
// exclusive prefix and its block total.
__global__ void __launch_bounds__(256)
k_scan1(const int* __restrict__ in, int n, int* __restrict__ loc, int* __restrict__ bsum) {
  __shared__ int sh[256];
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  int v[4], s = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    s += v[q];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int a = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += a;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - s;
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) loc[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = sh[255];
}

// Pass 2 (one workgroup): exclusive scan of the block totals; total[0] = sum.
__global__ void __launch_bounds__(1024) k_scan2(int* __restrict__ bsum, int nblk, int* __restrict__ total) {
  __shared__ int sh[1024];
  int carry = 0;
  for (int c0 = 0; c0 < nblk; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int v = i < nblk ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int a = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nblk) bsum[i] = carry + sh[threadIdx.x] - v;
    const int tot = sh[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) total[0] = carry;
}

// Pass 3: out[i] = loc[i] + bsum[block]; with `rows` set, a compaction:
// flagged entries get their rank (and rows[rank] = i), the others -1; ranks
// at or beyond `cap` are dropped (the host checks the total against it).
__global__ void __launch_bounds__(256)
k_scan3(const int* __restrict__ flag, int n, const int* __restrict__ loc, const int* __restrict__ bsum,
        int* __restrict__ out, int* __restrict__ rows, int cap) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int v = loc[i] + bsum[i / 1024];
  if (!rows) { out[i] = v; return; }
  if (flag[i] && v < cap) { out[i] = v; rows[v] = i; }
  else out[i] = -1;
}

// ---------------------------------------------------------------- active faces
// Finest level: every face a delta patch covers.
__global__ void __launch_bounds__(256)
k_mark0(int M, int N, const int* __restrict__ org, int* __restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * M) return;
  const int comp = t / M, NN = N * N;
  const int oi = org[2 * t], oj = org[2 * t + 1];
  for (int e = 0; e < 16; ++e)
    flag[comp * NN + wrapi(oj + (e >> 2), N) * N + wrapi(oi + (e & 3), N)] = 1;
}

// Level l+1: faces whose restriction stencil meets an active face of level l.
__global__ void __launch_bounds__(256)
k_mark_coarse(int Nc, const int* __restrict__ act_f, int* __restrict__ flag) {
  const int NNc = Nc * Nc, Nf = 2 * Nc, NNf = Nf * Nf, mf = Nf - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * NNc) return;
  const int comp = idx / NNc, rem = idx - comp * NNc;
  const int J = rem / Nc, I = rem - J * Nc;
  const int* a = act_f + comp * NNf;
  int any = 0;
  for (int d = -1; d <= 1; ++d)
    for (int e = 0; e <= 1; ++e) {
      const int x = comp == 0 ? 2 * I + d : 2 * I + e;
      const int y = comp == 0 ? 2 * J + e : 2 * J + d;
      any |= a[(y & mf) * Nf + (x & mf)] >= 0;
    }
  flag[idx] = any;
}

// ---------------------------------------------------------------- a5: elasticity windows
__device__ inline int wrap_half(int d, int N) {   // periodic offset into (-N/2, N/2]
  d = d & (N - 1);
  return d > N / 2 ? d - N : d;
}

// Finest level: row f of M_0 = -dt K S_0 L S^* (S_0 = W / h^2, S^* = W^T):
// kappa * sum over points k covering f of W_k(f) * sum_{k'} L_{k k'} W_{k'}.
// One wavefront per active row; lane t owns window entries t and t + 64 and
// gathers, for each point of the face's box list (ascending id) and each of
// its three fibre neighbours, the one patch entry that lands on it.  Every
// entry therefore sums its terms in (point, neighbour) order.  flags[0] |= 1
// if a nonzero falls outside the window.
__global__ void __launch_bounds__(256)
k_win0(PointView P, const int* __restrict__ rows, const int* __restrict__ nact, int maxact, double kappa,
       int reach, double* __restrict__ win, int* __restrict__ flags) {
  const int comp = blockIdx.y;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= maxact || row >= nact[comp]) return;
  const int N = P.N, msk = N - 1;
  const int f = rows[comp * maxact + row];
  const int i = f % N, j = f / N;
  const int box = (j / P.n) * P.nb + (i / P.n);
  const int* org = P.org + comp * P.M * 2;
  const double* wts = P.wts + (size_t)comp * P.M * IBMG_PATCH;
  const int q1 = lane + 64;
  const bool has1 = q1 < IBMG_WS;
  const int dx0 = lane % IBMG_WW - IBMG_WR, dy0 = lane / IBMG_WW - IBMG_WR;
  const int dx1 = q1 % IBMG_WW - IBMG_WR, dy1 = q1 / IBMG_WW - IBMG_WR;
  const bool in0 = dx0 >= -reach && dx0 <= reach && dy0 >= -reach && dy0 <= reach;
  const bool in1 = has1 && dx1 >= -reach && dx1 <= reach && dy1 >= -reach && dy1 <= reach;
  double acc0 = 0.0, acc1 = 0.0;
  int bad = 0;
  for (int q = P.box_start[box]; q < P.box_start[box + 1]; ++q) {
    const int k = P.box_list[q];
    const int di = (i - org[2 * k]) & msk, dj = (j - org[2 * k + 1]) & msk;
    if (di >= 4 || dj >= 4) continue;
    const double bk = kappa * wts[k * IBMG_PATCH + dj * 4 + di];
    const int nbk[3] = {P.prev[k], k, P.next[k]};
    const double lc[3] = {1.0, -2.0, 1.0};
    for (int s = 0; s < 3; ++s) {
      const int kk = nbk[s];
      const int oi = org[2 * kk], oj = org[2 * kk + 1];
      const double* wk = wts + kk * IBMG_PATCH;
      const double bl = bk * lc[s];
      if (in0) {
        const int ex = (i + dx0 - oi) & msk, ey = (j + dy0 - oj) & msk;
        if (ex < 4 && ey < 4 && wrap_half(oi + ex - i, N) == dx0 && wrap_half(oj + ey - j, N) == dy0)
          acc0 += bl * wk[ey * 4 + ex];
      }
      if (in1) {
        const int ex = (i + dx1 - oi) & msk, ey = (j + dy1 - oj) & msk;
        if (ex < 4 && ey < 4 && wrap_half(oi + ex - i, N) == dx1 && wrap_half(oj + ey - j, N) == dy1)
          acc1 += bl * wk[ey * 4 + ex];
      }
      if (lane < 16) {   // does patch entry `lane` fall outside the window?
        const double val = bl * wk[lane];
        const int dx = wrap_half(oi + (lane & 3) - i, N), dy = wrap_half(oj + (lane >> 2) - j, N);
        if ((dx < -reach || dx > reach || dy < -reach || dy > reach) && val != 0.0) bad = 1;
      }
    }
  }
  double* o = win + ((size_t)comp * maxact + row) * IBMG_WS;
  o[lane] = acc0;
  if (has1) o[q1] = acc1;
  if (bad) atomicOr(flags, 1);
}

// Level l -> l+1: row F of R M_l P.  For each fine row f of the restriction
// stencil of F (weight rw) and each window entry g = f + d of that row, the
// coefficient goes to the coarse faces G of the bilinear prolongation stencil
// of g (weight pw) at offset G - F, all on unwrapped indices.  One wavefront
// per coarse row; lane t owns coarse entries t and t + 64 and gathers the
// fine entries g whose prolongation reaches it (normal index 2G-1..2G+1,
// tangential 2G-1..2G+2), fine rows in stencil order and g in row-major
// order within each.  flags[0] |= 2 if a contribution falls outside the
// coarse window.
// With walls the transfers are the walled ones: coarse wall faces (normal
// index 0, or Nc for the far wall) and faces outside the domain neither
// restrict nor receive (their row and column of R M P are zero), fine faces
// outside the domain do not exist, and the fine row next to a wall parallel
// to the face prolongs from its coarse row with weight 1/2 (the coarse
// field's ghost across the wall is -e).
__device__ inline double win_coarse_entry(int comp, int FX, int FY, int ox, int oy, const int* __restrict__ af,
                                          const double* __restrict__ win_f, int maxact_f, int reach_f, int Nf,
                                          int walls) {
  const int mf = Nf - 1, Nc = Nf / 2;
  const double wr[3] = {0.125, 0.25, 0.125};
  const int GX = FX + ox, GY = FY + oy;
  const int gn0 = 2 * (comp == 0 ? GX : GY), gt0 = 2 * (comp == 0 ? GY : GX);
  if (walls) {
    const int Fn = comp == 0 ? FX : FY, Gn = comp == 0 ? GX : GY, Gt = comp == 0 ? GY : GX;
    if (Fn == 0 || Gn <= 0 || Gn >= Nc || Gt < 0 || Gt >= Nc) return 0.0;
  }
  double acc = 0.0;
  for (int d = -1; d <= 1; ++d)
    for (int e = 0; e <= 1; ++e) {
      const int fx = comp == 0 ? 2 * FX + d : 2 * FX + e;
      const int fy = comp == 0 ? 2 * FY + e : 2 * FY + d;
      const int ar = af[(fy & mf) * Nf + (fx & mf)];
      if (ar < 0) continue;
      const double rw = wr[d + 1];
      const double* cw = win_f + ((size_t)comp * maxact_f + ar) * IBMG_WS;
      // g in row-major (gy outer) order
      const int ylo = comp == 0 ? gt0 - 1 : gn0 - 1, yhi = comp == 0 ? gt0 + 2 : gn0 + 1;
      const int xlo = comp == 0 ? gn0 - 1 : gt0 - 1, xhi = comp == 0 ? gn0 + 1 : gt0 + 2;
      for (int gy = ylo; gy <= yhi; ++gy) {
        const int dy = gy - fy;
        if (dy < -reach_f || dy > reach_f) continue;
        for (int gx = xlo; gx <= xhi; ++gx) {
          const int dx = gx - fx;
          if (dx < -reach_f || dx > reach_f) continue;
          const double val = rw * cw[(dy + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
          if (val == 0.0) continue;
          const int gn = comp == 0 ? gx : gy, gt = comp == 0 ? gy : gx;
          const double wn = gn == gn0 ? 1.0 : 0.5;
          double wt = (gt == gt0 || gt == gt0 + 1) ? 0.75 : 0.25;
          if (walls) {
            if (gn <= 0 || gn >= Nf || gt < 0 || gt >= Nf) continue;
            if (gt == 0 || gt == Nf - 1) wt = 0.5;
          }
          acc += val * wn * wt;
        }
      }
    }
  return acc;
}

__global__ void __launch_bounds__(256)
k_win_coarse(int Nc, const int* __restrict__ act_f, const double* __restrict__ win_f, int maxact_f, int reach_f,
             const int* __restrict__ rows, const int* __restrict__ nact, int maxact, int reach,
             double* __restrict__ win, int* __restrict__ flags, int walls) {
  const int comp = blockIdx.y;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= maxact || row >= nact[comp]) return;
  const int Nf = 2 * Nc, NNf = Nf * Nf, mf = Nf - 1;
  const int F = rows[comp * maxact + row];
  const int FX = F % Nc, FY = F / Nc;
  const int* af = act_f + comp * NNf;
  const int q1 = lane + 64;
  const bool has1 = q1 < IBMG_WS;
  const int dx0 = lane % IBMG_WW - IBMG_WR, dy0 = lane / IBMG_WW - IBMG_WR;
  const int dx1 = q1 % IBMG_WW - IBMG_WR, dy1 = q1 / IBMG_WW - IBMG_WR;
  double acc0 = 0.0, acc1 = 0.0;
  if (dx0 >= -reach && dx0 <= reach && dy0 >= -reach && dy0 <= reach)
    acc0 = win_coarse_entry(comp, FX, FY, dx0, dy0, af, win_f, maxact_f, reach_f, Nf, walls);
  if (has1 && dx1 >= -reach && dx1 <= reach && dy1 >= -reach && dy1 <= reach)
    acc1 = win_coarse_entry(comp, FX, FY, dx1, dy1, af, win_f, maxact_f, reach_f, Nf, walls);
  double* o = win + ((size_t)comp * maxact + row) * IBMG_WS;
  o[lane] = acc0;
  if (has1) o[q1] = acc1;
  // window check: every nonzero fine entry's prolongation targets
  int bad = 0;
  for (int d = -1; d <= 1; ++d)
    for (int e = 0; e <= 1; ++e) {
      const int fx = comp == 0 ? 2 * FX + d : 2 * FX + e;
      const int fy = comp == 0 ? 2 * FY + e : 2 * FY + d;
      const int ar = af[(fy & mf) * Nf + (fx & mf)];
      if (ar < 0) continue;
      const double* cw = win_f + ((size_t)comp * maxact_f + ar) * IBMG_WS;
      for (int q = lane; q < IBMG_WS; q += 64) {
        const int dx = q % IBMG_WW - IBMG_WR, dy = q / IBMG_WW - IBMG_WR;
        if (dx < -reach_f || dx > reach_f || dy < -reach_f || dy > reach_f || cw[q] == 0.0) continue;
        const int gn = comp == 0 ? fx + dx : fy + dy, gt = comp == 0 ? fy + dy : fx + dx;
        const int n0 = gn >> 1, n1 = (gn + 1) >> 1;               // coarse normal indices reached
        const int t0 = (gt >> 1) - ((gt & 1) == 0 ? 1 : 0), t1 = (gt >> 1) + ((gt & 1) == 0 ? 0 : 1);
        const int Fn = comp == 0 ? FX : FY, Ft = comp == 0 ? FY : FX;
        if (n0 - Fn < -reach || n1 - Fn > reach || t0 - Ft < -reach || t1 - Ft > reach) bad = 1;
      }
    }
  if (bad) atomicOr(flags, 2);
}

// Per-colour lists of the active rows (four colours): a face lies in the
// box that holds it and, on a box edge across its normal, also in the
// neighbour before it (periodic index); the two boxes differ in colour, so
// each list holds a row at most once.  The order within a list depends on
// the atomics; each row is evaluated on its own, so the results do not.
__global__ void __launch_bounds__(256)
k_colour_rows(int N, int n, int nb, const int* __restrict__ rows, const int* __restrict__ nact, int maxact,
              int* __restrict__ crow, int* __restrict__ ncrow) {
  const int comp = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= min(nact[comp], maxact)) return;
  const int f = rows[comp * maxact + r];
  const int i = f % N, j = f / N;
  const int a = comp == 0 ? i : j, t = comp == 0 ? j : i;   // along the normal, along the tangent
  const int ba[2] = {a / n, (a / n + nb - 1) % nb};
  const int nba = (a % n == 0) ? 2 : 1;
  for (int q = 0; q < nba; ++q) {
    const int bx = comp == 0 ? ba[q] : t / n, by = comp == 0 ? t / n : ba[q];
    const int c = (bx & 1) | ((by & 1) << 1);
    const int slot = atomicAdd(&ncrow[c * 2 + comp], 1);
    crow[(size_t)(c * 2 + comp) * maxact + slot] = r;
  }
}

// ---------------------------------------------------------------- boxes with elastic rows
// A box takes its own inverse if one of its faces has elastic rows (act
// given) or, with walls, if it touches a wall (its block differs from the
// interior boxes' shared one).
__global__ void __launch_bounds__(256)
k_box_flag(int N, int n, int nb, const int* __restrict__ act, int walls, int* __restrict__ flag) {
  const int box = blockIdx.x * blockDim.x + threadIdx.x;
  if (box >= nb * nb) return;
  const int bx = box % nb, by = box / nb, NN = N * N;
  int any = walls && (bx == 0 || by == 0 || bx == nb - 1 || by == nb - 1);
  for (int lj = 0; act && lj <= n && !any; ++lj)
    for (int li = 0; li <= n; ++li) {
      if (lj < n) any |= act[wrapi(by * n + lj, N) * N + wrapi(bx * n + li, N)] >= 0;           // u
      if (li < n) any |= act[NN + wrapi(by * n + lj, N) * N + wrapi(bx * n + li, N)] >= 0;      // v
    }
  flag[box] = any;
}

// Block-wide exclusive scan helper (1024 threads).
__device__ inline int block_excl_scan(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int a = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  total = sh[1023];
  const int incl = sh[tid];
  __syncthreads();
  return incl - v;
}

// Number the flagged boxes colour class by colour class (see colour_box),
// in the order a sweep visits them (nb >= 2, even).  ib_boxes[idx] = box id;
// info[c] = count of colour c; info[4] = total.
__global__ void __launch_bounds__(1024)
k_ib_index(int nb, int ncol, const int* __restrict__ flagb, int* __restrict__ ib_index, int* __restrict__ ib_boxes,
           int* __restrict__ info) {
  __shared__ int sh[1024];
  const int per = colour_count(ncol, nb);
  int base = 0;
  for (int c = 0; c < ncol; ++c) {
    int cbase = base;
    for (int c0 = 0; c0 < per; c0 += 1024) {
      const int q = c0 + threadIdx.x;
      int box = 0, flag = 0;
      if (q < per) {
        int bx, by;
        colour_box(q, c, ncol, nb, bx, by);
        box = by * nb + bx;
        flag = flagb[box] ? 1 : 0;
      }
      int total;
      const int ex = block_excl_scan(flag, sh, total);
      if (q < per) {
        ib_index[box] = flag ? cbase + ex : -1;
        if (flag) ib_boxes[cbase + ex] = box;
      }
      cbase += total;
    }
    if (threadIdx.x == 0) info[c] = cbase - base;
    base = cbase;
  }
  if (threadIdx.x == 0) {
    for (int c = ncol; c < 4; ++c) info[c] = 0;
    info[4] = base;
  }
}

// ---------------------------------------------------------------- a6: box blocks
// Assemble A_l[box, box] (Stokes stencil restricted to the box plus the
// elasticity rows' window entries whose column lies in the box) into an LDS
// buffer with leading dimension ld.
__device__ void assemble_box(const LevelView<double>& L, int bx, int by, bool with_ib, double* a, int ld) {
  const int n = L.n, N = L.N, nd = L.ndof, NN = N * N;
  for (int r = threadIdx.x; r < nd; r += blockDim.x) {
    int comp, i, j;
    box_dof(r, bx, by, n, N, comp, i, j);
    double* row = a + (size_t)r * ld;
    const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
    int col;
    if (L.walls) {   // the walled rows of stokes_row_walls
      if (comp < 2) {
        const int an = comp == 0 ? i : j, at = comp == 0 ? j : i;
        if (an == 0) {   // wall face: identity row
          row[r] += 1.0;
          continue;
        }
        const int ghosts = (at + 1 < N ? 0 : 1) + (at > 0 ? 0 : 1);
        row[r] += L.c + (4.0 + ghosts) * L.muh2;
        // (normal +1, normal -1, tangent +1, tangent -1) neighbours inside the walls
        const bool ok[4] = {an + 1 < N, an - 1 > 0, at + 1 < N, at > 0};
        const int nbi[4] = {comp == 0 ? i + 1 : i, comp == 0 ? i - 1 : i, comp == 0 ? i : i + 1, comp == 0 ? i : i - 1};
        const int nbj[4] = {comp == 0 ? j : j + 1, comp == 0 ? j : j - 1, comp == 0 ? j + 1 : j, comp == 0 ? j - 1 : j};
        for (int q = 0; q < 4; ++q)
          if (ok[q] && (col = box_local(comp, nbi[q], nbj[q], bx, by, n, N)) >= 0) row[col] -= L.muh2;
        if ((col = box_local(2, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if ((col = box_local(2, comp == 0 ? i - 1 : i, comp == 0 ? j : j - 1, bx, by, n, N)) >= 0)
          row[col] -= L.invh;
        // with walls a box may take its own inverse without elastic rows
        // (a box along a wall, or no structure at all): act is then absent
        const int ar = (with_ib && L.act) ? L.act[comp * NN + j * N + i] : -1;
        if (ar >= 0) {
          const double* cw = L.win + ((size_t)comp * L.maxact + ar) * IBMG_WS;
          for (int dy = -L.reach; dy <= L.reach; ++dy)
            for (int dx = -L.reach; dx <= L.reach; ++dx)
              if ((col = box_local(comp, wrapi(i + dx, N), wrapi(j + dy, N), bx, by, n, N)) >= 0)
                row[col] += cw[(dy + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
        }
      } else {
        if (i + 1 < N && (col = box_local(0, i + 1, j, bx, by, n, N)) >= 0) row[col] -= L.invh;
        if (i > 0 && (col = box_local(0, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if (j + 1 < N && (col = box_local(1, i, j + 1, bx, by, n, N)) >= 0) row[col] -= L.invh;
        if (j > 0 && (col = box_local(1, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
      }
      continue;
    }
    if (comp < 2) {
      row[r] += L.c + 4.0 * L.muh2;
      const int nbi[4] = {ip, im, i, i}, nbj[4] = {j, j, jp, jm};
      for (int q = 0; q < 4; ++q)
        if ((col = box_local(comp, nbi[q], nbj[q], bx, by, n, N)) >= 0) row[col] -= L.muh2;
      if (comp == 0) {
        if ((col = box_local(2, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if ((col = box_local(2, im, j, bx, by, n, N)) >= 0) row[col] -= L.invh;
      } else {
        if ((col = box_local(2, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
        if ((col = box_local(2, i, jm, bx, by, n, N)) >= 0) row[col] -= L.invh;
      }
      const int ar = (with_ib && L.act) ? L.act[comp * NN + j * N + i] : -1;
      if (ar >= 0) {
        const double* cw = L.win + ((size_t)comp * L.maxact + ar) * IBMG_WS;
        for (int dy = -L.reach; dy <= L.reach; ++dy)
          for (int dx = -L.reach; dx <= L.reach; ++dx)
            if ((col = box_local(comp, wrapi(i + dx, N), wrapi(j + dy, N), bx, by, n, N)) >= 0)
              row[col] += cw[(dy + IBMG_WR) * IBMG_WW + dx + IBMG_WR];
      }
    } else {
      if ((col = box_local(0, ip, j, bx, by, n, N)) >= 0) row[col] -= L.invh;
      if ((col = box_local(0, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
      if ((col = box_local(1, i, jp, bx, by, n, N)) >= 0) row[col] -= L.invh;
      if ((col = box_local(1, i, j, bx, by, n, N)) >= 0) row[col] += L.invh;
    }
  }
}

// Block 0: the plain box (Stokes only, shared by every box without elastic
// rows).  Block 1 + q: box ib_boxes[q].  Inverses are written column-major.
// Level of block blk of a multi-level factor launch (uniform per block).
__device__ inline int factor_level(const ibmg::BoxFactorLevels& F, int blk) {
  int l = 0;
  while (l + 1 < F.nl && blk >= F.first[l + 1]) ++l;
  return l;
}

__global__ void __launch_bounds__(128) k_box_factor(ibmg::BoxFactorLevels F) {
  __shared__ double a[IBMG_MAX_NDOF * 2 * IBMG_MAX_NDOF];
  __shared__ double colk[IBMG_MAX_NDOF];
  __shared__ int piv;
  __shared__ double pval;
  const int lv = factor_level(F, blockIdx.x), blk = blockIdx.x - F.first[lv];
  const LevelView<double>& L = F.v[lv];
  double* ainv_plain = F.ainv_plain[lv];
  float* ainv_plain_f = F.ainv_plain_f[lv];
  const int nd = L.ndof, ld = 2 * nd;
  const bool plain = blk == 0;
  int bx = 0, by = 0;
  if (!plain) {
    const int box = F.ib_boxes[lv][blk - 1];
    bx = box % L.nb;
    by = box / L.nb;
  } else if (L.walls && L.nb >= 3) {   // the shared block is an interior box's
    bx = 1;
    by = 1;
  }
  for (int idx = threadIdx.x; idx < nd * ld; idx += blockDim.x) {
    const int i = idx / ld, c = idx - i * ld;
    a[idx] = (c == nd + i) ? 1.0 : 0.0;
  }
  __syncthreads();
  assemble_box(L, bx, by, !plain, a, ld);
  __syncthreads();
  gauss_jordan_cols(a, nd, ld, colk, &piv, &pval);
  double* out = plain ? ainv_plain : F.ainv_ib[lv] + (size_t)(blk - 1) * nd * nd;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) {
    const int r = idx / nd, c = idx - r * nd;
    const double v = a[r * ld + nd + c];
    out[c * nd + r] = v;
    if (plain && ainv_plain_f) ainv_plain_f[c * nd + r] = (float)v;
  }
}

// Blocks of 8 x 8 boxes (208 unknowns): assembled row-major into their own
// output slot, then inverted in registers (gj_reg.h) and written back
// column-major over it.  Same block numbering as k_box_factor.
__global__ void __launch_bounds__(kGjLanes) k_box_factor_big(ibmg::BoxFactorLevels F) {
  __shared__ GjScratch S;
  const int lv = factor_level(F, blockIdx.x), blk = blockIdx.x - F.first[lv];
  const LevelView<double>& L = F.v[lv];
  const int nd = L.ndof;
  const bool plain = blk == 0;
  int bx = 0, by = 0;
  if (!plain) {
    const int box = F.ib_boxes[lv][blk - 1];
    bx = box % L.nb;
    by = box / L.nb;
  } else if (L.walls && L.nb >= 3) {
    bx = 1;
    by = 1;
  }
  double* slot = plain ? F.ainv_plain[lv] : F.ainv_ib[lv] + (size_t)(blk - 1) * nd * nd;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) slot[idx] = 0.0;
  __syncthreads();
  assemble_box(L, bx, by, !plain, slot, nd);
  __syncthreads();
  float* f32 = plain ? F.ainv_plain_f[lv] : nullptr;
  gauss_jordan_regs(
      nd, S, [&](int i, int j) { return slot[(size_t)i * nd + j]; },
      [&](int r, int c, double v) {
        slot[(size_t)c * nd + r] = v;
        if (f32) f32[(size_t)c * nd + r] = (float)v;
      });
}

// Assembled (not inverted) block of one box, row-major, for inspection
// (blocks larger than the LDS buffer are assembled in place in out).
__global__ void __launch_bounds__(256)
k_box_matrix(LevelView<double> L, int bx, int by, double* __restrict__ out) {
  __shared__ double a[IBMG_MAX_NDOF * IBMG_MAX_NDOF];
  const int nd = L.ndof;
  double* buf = nd <= IBMG_MAX_NDOF ? a : out;
  for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) buf[idx] = 0.0;
  __syncthreads();
  assemble_box(L, bx, by, L.act != nullptr, buf, nd);
  __syncthreads();
  if (buf == a)
    for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) out[idx] = a[idx];
}

// ---------------------------------------------------------------- launchers
namespace ibmg {

void launch_fiber_force(hipStream_t s, int M, const int* prev, const int* next, double K,
                        const double* X, double* G) {
  if (M > 0) k_fiber_force<<<nblk(M), 256, 0, s>>>(M, prev, next, K, X, G);
}

void launch_weights0(hipStream_t s, int M, int N, int kind, const double* X, int* org, double* w) {
  if (M > 0) k_weights0<<<nblk(2 * (size_t)M), 256, 0, s>>>(M, N, kind, X, org, w);
}

void launch_scan(hipStream_t s, const int* in, int n, int* out, int* rows, int cap, int* total, int* loc,
                 int* bsum) {
  const int nb1 = (n + 1023) / 1024;
  k_scan1<<<nb1, 256, 0, s>>>(in, n, loc, bsum);
  k_scan2<<<1, 1024, 0, s>>>(bsum, nb1, total);
  k_scan3<<<nblk(n), 256, 0, s>>>(in, n, loc, bsum, out, rows, cap);
}

void launch_box_lists(hipStream_t s, const PointView& P, int* cnt, int* start, int* cursor, int* list,
                      int max_list, int* total, int* loc, int* bsum) {
  const int nbox = P.nb * P.nb;
  k_fill_i32<<<nblk(nbox + 1), 256, 0, s>>>(cnt, nbox + 1, 0);
  k_fill_i32<<<nblk(nbox), 256, 0, s>>>(cursor, nbox, 0);
  if (P.M > 0) k_box_count<<<nblk(P.M), 256, 0, s>>>(P.M, P.org, P.n, P.N, P.nb, cnt);
  // start[0..nbox] = exclusive scan of cnt[0..nbox] (cnt[nbox] = 0, so start[nbox] = total)
  launch_scan(s, cnt, nbox + 1, start, nullptr, 0, total, loc, bsum);
  if (P.M > 0) {
    k_box_fill<<<nblk(P.M), 256, 0, s>>>(P.M, P.org, P.n, P.N, P.nb, start, cursor, list, max_list);
    k_box_sort<<<nbox, kSortLanes, 0, s>>>(nbox, start, list, max_list);
  }
}

void launch_active(hipStream_t s, int level, int M, int N, const int* org, const int* act_fine, int* flag,
                   int* act, int* rows, int* nact, int maxact, int* loc, int* bsum) {
  const int NN = N * N;
  k_fill_i32<<<nblk(2 * (size_t)NN), 256, 0, s>>>(flag, 2 * NN, 0);
  if (level == 0) {
    if (M > 0) k_mark0<<<nblk(2 * (size_t)M), 256, 0, s>>>(M, N, org, flag);
  } else {
    k_mark_coarse<<<nblk(2 * (size_t)NN), 256, 0, s>>>(N, act_fine, flag);
  }
  for (int c = 0; c < 2; ++c)
    launch_scan(s, flag + c * NN, NN, act + c * NN, rows + c * maxact, maxact, nact + c, loc, bsum);
}

void launch_windows0(hipStream_t s, const PointView& P, const int* rows, const int* nact, int maxact, double kappa,
                     int reach, double* win, int* flags) {
  dim3 g((unsigned)((maxact + 3) / 4), 2);
  k_win0<<<g, 256, 0, s>>>(P, rows, nact, maxact, kappa, reach, win, flags);
}

void launch_windows_coarse(hipStream_t s, int Nc, const int* act_f, const double* win_f, int maxact_f, int reach_f,
                           const int* rows, const int* nact, int maxact, int reach, double* win, int* flags,
                           int walls) {
  dim3 g((unsigned)((maxact + 3) / 4), 2);
  k_win_coarse<<<g, 256, 0, s>>>(Nc, act_f, win_f, maxact_f, reach_f, rows, nact, maxact, reach, win, flags, walls);
}

void launch_colour_rows(hipStream_t s, int N, int n, int nb, const int* rows, const int* nact, int maxact, int* crow,
                        int* ncrow) {
  k_fill_i32<<<1, 256, 0, s>>>(ncrow, 8, 0);
  k_colour_rows<<<dim3((unsigned)((maxact + 255) / 256), 2), 256, 0, s>>>(N, n, nb, rows, nact, maxact, crow, ncrow);
}

void launch_box_classes(hipStream_t s, int N, int n, int nb, int ncol, const int* act, int walls, int* flag,
                        int* ib_index, int* ib_boxes, int* info) {
  if (act || walls) k_box_flag<<<nblk(nb * nb), 256, 0, s>>>(N, n, nb, act, walls, flag);
  else k_fill_i32<<<nblk(nb * nb), 256, 0, s>>>(flag, nb * nb, 0);
  k_ib_index<<<1, 1024, 0, s>>>(nb, ncol, flag, ib_index, ib_boxes, info);
}

void launch_box_factor(hipStream_t s, const BoxFactorLevels& F) {
  const int nblocks = F.first[F.nl];
  if (F.nl <= 0 || nblocks <= 0) return;
  if (F.v[0].ndof <= IBMG_MAX_NDOF) k_box_factor<<<nblocks, 128, 0, s>>>(F);
  else k_box_factor_big<<<nblocks, kGjLanes, 0, s>>>(F);
}

void launch_box_matrix(hipStream_t s, const LevelView<double>& L, int bx, int by, double* out) {
  k_box_matrix<<<1, 256, 0, s>>>(L, bx, by, out);
}

}  // namespace ibmg
