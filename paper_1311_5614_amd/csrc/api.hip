// Host side of the C ABI (include/ibmg.h): validation, workspace layout, the
// per-step setup sequence, the V-cycle schedule (Algorithm 1), FGMRES and the
// implicit time step.  Every arithmetic step runs in the gfx950 kernels of
// ib_setup.hip, mg.hip, dense.hip and krylov.hip; the host only sequences
// launches on the handle's stream and reads back scalars for control flow.
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

namespace ibmg {

void take(size_t& cur, Buf& b, size_t bytes) {
  cur = (cur + 255) & ~(size_t)255;
  b.off = cur;
  b.bytes = bytes;
  cur += bytes;
}

int boxes_per_point(int n) {
  const int a = (4 + n - 1) / n + 2;
  return a * a;
}

int window_reach(int level) { return level == 0 ? IBMG_WR : (level == 1 ? 4 : 3); }

void layout(ibmg_handle* h) {
  size_t cur = 0;
  // V-cycle vectors are sized for FP64 also on an FP32 handle: a stalled FP32
  // solve continues with the FP64 V-cycle on the same buffers
  const size_t rs = sizeof(double);
  const int M = h->M, bpp = boxes_per_point(h->n);
  h->ndof = 2 * h->n * (h->n + 1) + h->n * h->n;
  const size_t nd2 = (size_t)h->ndof * h->ndof;
  const bool ib = M > 0;
  for (int l = 0; l < h->levels; ++l) {
    LevelBufs& B = h->L[l];
    B.N = h->N >> l;
    B.nb = B.N / h->n;
    B.reach = window_reach(l);
    const size_t NN = (size_t)B.N * B.N;
    if (l > 0 || h->prec == IBMG_FP32) {
      take(cur, B.w, 3 * NN * rs);
      take(cur, B.b, 3 * NN * rs);
    }
    take(cur, B.r, 3 * NN * rs);
    if (ib) {
      // each point covers 16 faces per component on the finest level; each
      // active face of a level activates at most two faces of the next
      B.maxact = (int)std::max<size_t>(1, std::min<size_t>(NN, (size_t)16 * M << l));
      take(cur, B.act, 2 * NN * sizeof(int));
      take(cur, B.rows, 2 * (size_t)B.maxact * sizeof(int));
      take(cur, B.nact, 2 * sizeof(int));
      take(cur, B.win, 2 * (size_t)B.maxact * IBMG_WS * sizeof(double));
      if (h->prec == IBMG_FP32) take(cur, B.winf, 2 * (size_t)B.maxact * IBMG_WS * sizeof(float));
      take(cur, B.yib, 2 * NN * sizeof(double));
      if (l < h->levels - 1 && phase_fusable(h->ncol_l[l], h->n)) {
        take(cur, B.crow, 8 * (size_t)B.maxact * sizeof(int));
        take(cur, B.ncrow, 8 * sizeof(int));
      }
    }
    if (l < h->levels - 1) {
      const size_t nbox = (size_t)B.nb * B.nb;
      take(cur, B.ib_index, nbox * sizeof(int));
      take(cur, B.ib_boxes, nbox * sizeof(int));
      take(cur, B.boxflag, nbox * sizeof(int));
      take(cur, B.info, 8 * sizeof(int));
      take(cur, B.ainv_plain, nd2 * sizeof(double));
      take(cur, B.ainv_plain_f, nd2 * sizeof(float));
      // boxes with elastic rows, plus with walls the 4 (nb - 1) boxes along them
      B.max_ib = (int)std::min<size_t>(nbox, (ib ? (size_t)M * bpp : 0) + (h->walls ? 4 * (size_t)B.nb : 0));
      take(cur, B.ainv_ib, std::max<size_t>(1, (size_t)B.max_ib) * nd2 * sizeof(double));
    }
  }
  const size_t N0 = (size_t)h->N * h->N, nbox0 = (size_t)h->L[0].nb * h->L[0].nb;
  const int Nc = h->N >> (h->levels - 1);
  h->nr = 3 * Nc * Nc + 1;
  const size_t nr = h->nr;
  take(cur, h->aug, nr * 2 * nr * sizeof(double));
  take(cur, h->cm, nr * kPW * sizeof(double));
  take(cur, h->cpiv, nr * sizeof(int));
  take(cur, h->crowpos, nr * sizeof(int));
  take(cur, h->cused, nr * sizeof(int));
  take(cur, h->cY, (size_t)kPW * 2 * nr * sizeof(double));
  take(cur, h->cainv, nr * nr * sizeof(double));
  const size_t Mx = std::max(1, M);
  take(cur, h->X0, 2 * Mx * sizeof(double));
  take(cur, h->G, 2 * Mx * sizeof(double));
  take(cur, h->U, 2 * Mx * sizeof(double));
  take(cur, h->prev_d, Mx * sizeof(int));
  take(cur, h->next_d, Mx * sizeof(int));
  take(cur, h->org, 4 * Mx * sizeof(int));
  take(cur, h->wts, 2 * Mx * IBMG_PATCH * sizeof(double));
  take(cur, h->cnt, (nbox0 + 1) * sizeof(int));
  take(cur, h->start, (nbox0 + 1) * sizeof(int));
  take(cur, h->cursor, nbox0 * sizeof(int));
  h->max_list = std::max(1, M * bpp);
  take(cur, h->list, (size_t)h->max_list * sizeof(int));
  take(cur, h->ltotal, 4 * sizeof(int));
  const size_t scan_n = std::max(2 * N0, nbox0 + 1);
  take(cur, h->flag, scan_n * sizeof(int));
  take(cur, h->loc, scan_n * sizeof(int));
  take(cur, h->bsum, (scan_n / 1024 + 2) * sizeof(int));
  take(cur, h->meta, 8 * sizeof(int));
  const size_t n0 = h->n0(), m = h->mb;
  take(cur, h->V, (m + 1) * n0 * sizeof(double));
  take(cur, h->Z, m * n0 * sizeof(double));
  take(cur, h->H, (m + 1) * (m + 1) * sizeof(double));
  take(cur, h->g, (m + 2) * sizeof(double));
  take(cur, h->cs, (m + 1) * sizeof(double));
  take(cur, h->sn, (m + 1) * sizeof(double));
  take(cur, h->y, (m + 1) * sizeof(double));
  take(cur, h->hc, 2 * (m + 2) * sizeof(double));
  take(cur, h->flags, 8 * sizeof(double));
  take(cur, h->scal, 16 * sizeof(double));
  // product passes (two vectors per pass in the delayed form) and the
  // per-workgroup norm shares of the delayed form's update pass
  take(cur, h->partial, std::max((size_t)kDotBlocks * 2 * (m + 2), (size_t)nblk(n0)) * sizeof(double));
  take(cur, h->bvec, n0 * sizeof(double));
  take(cur, h->xvec, n0 * sizeof(double));
  take(cur, h->rvec, n0 * sizeof(double));
  take(cur, h->xbest, n0 * sizeof(double));
  if (h->prec == IBMG_FP32) {
    take(cur, h->w0f, n0 * sizeof(float));
    take(cur, h->b0f, n0 * sizeof(float));
  } else {
    take(cur, h->w0g, n0 * sizeof(double));
    take(cur, h->b0g, n0 * sizeof(double));
  }
  h->need = cur + 256;
}

}  // namespace ibmg

namespace {

using namespace ibmg;

int sync(ibmg_handle* h) {
  IBMG_HIP(hipStreamSynchronize(h->stream));
  return IBMG_OK;
}

int read_doubles(ibmg_handle* h, const double* dev, double* host, int n) {
  IBMG_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  IBMG_HIP(hipStreamSynchronize(h->stream));
  return IBMG_OK;
}

// ---------------------------------------------------------------- V-cycle schedule

// One colour phase (residual + elastic rows, then box solves), with the box
// kernel timed by events when timing is on.  from_zero: the iterate is zero
// (the first phase of a level's pre-smoothing: Algorithm 1 starts the
// correction at zero), so the residual is b itself and the elastic term is
// zero; the boxes read b directly and no residual pass is launched.
template <typename T>
void phase_timed(ibmg_handle* h, const LevelView<T>& v, int l, const T* b, T* w, T* r, int colour,
                 bool from_zero) {
  LevelView<T> vb = v;
  // four colours: the boxes form their own Stokes residuals, one launch per
  // phase (plus the elastic-row pass); otherwise the residual pass first
  const bool fused = !from_zero && phase_fusable(v.ncol, v.n);
  if (from_zero) vb.yib = nullptr;
  else if (!fused) launch_res<T>(h->stream, v, b, w, r, h->has_ib);
  const bool t = h->timing && h->ev_used + 2 <= (int)h->ev.size();
  if (t) (void)hipEventRecord(h->ev[h->ev_used], h->stream);
  if (fused) launch_phase_fused<T>(h->stream, v, b, w, colour, h->own_boxes());
  else launch_box<T>(h->stream, vb, from_zero ? b : r, w, colour, h->own_boxes());
  if (t) {
    (void)hipEventRecord(h->ev[h->ev_used + 1], h->stream);
    // algorithmic bytes of one box launch: per unknown of the colour's boxes
    // read r and w, write w; the shared inverse once; each FP64 inverse of a
    // box with elastic rows once
    const double boxes = colour_count(v.ncol, v.nb);
    double bytes = boxes * v.ndof * 3.0 * sizeof(T) + (double)v.ndof * v.ndof * sizeof(T);
    if (h->own_boxes()) bytes += (double)h->n_ib[l][colour] * v.ndof * v.ndof * sizeof(double);
    h->ev_bytes[h->ev_used / 2] = bytes;
    h->ev_used += 2;
  }
}

template <typename T>
void sweep(ibmg_handle* h, const LevelView<T>& v, int l, const T* b, T* w, T* r, bool from_zero = false) {
  for (int c = 0; c < v.ncol; ++c) phase_timed<T>(h, v, l, b, w, r, c, from_zero && c == 0);
}

// z = MGV(0, r) on level 0 (Algorithm 1), vectors in precision T.
template <typename T>
void vcycle(ibmg_handle* h, const T* b0, T* w0, bool w0_zero = false) {
  const int Lv = h->levels;
  hipStream_t s = h->stream;
  T* w[IBMG_MAX_LEVELS];
  const T* b[IBMG_MAX_LEVELS];
  T* r[IBMG_MAX_LEVELS];
  LevelView<T> v[IBMG_MAX_LEVELS];
  for (int l = 0; l < Lv; ++l) {
    v[l] = view<T>(h, l);
    w[l] = l == 0 ? w0 : h->p<T>(h->L[l].w);
    b[l] = l == 0 ? b0 : h->p<T>(h->L[l].b);
    r[l] = h->p<T>(h->L[l].r);
  }
  // levels ls.. (at most tail_max cells per side, plus the coarsest) run in
  // one LDS-resident workgroup; a tail of the coarsest level alone is its
  // matrix-vector product, spread over the grid
  const int ls = tail_start(h);
  if (ls > 0 && !w0_zero) {   // w0_zero: the caller's input pass has cleared w[0]
    const size_t n3 = 3 * (size_t)v[0].N * v[0].N;
    k_fill<T><<<nblk(n3), 256, 0, s>>>(w[0], n3, T(0));
  }
  for (int l = 0; l < ls; ++l) {
    // w[l] is zero here (cleared above, or by the restriction into level l)
    for (int q = 0; q < h->nu1; ++q) sweep<T>(h, v[l], l, b[l], w[l], r[l], q == 0);
    // Stokes residual and the elastic term in one pass; the restriction
    // subtracts the elastic term (also zeroes w[l+1])
    launch_res<T>(s, v[l], b[l], w[l], r[l], h->has_ib);
    launch_restrict<T>(s, v[l].N, r[l], h->p<T>(h->L[l + 1].b), w[l + 1], h->has_ib ? v[l].yib : nullptr,
                       h->walls);
  }
  if (ls == Lv - 1)
    launch_coarse_apply<T>(s, h->p<double>(h->cainv), h->nr, b[ls], w[ls]);
  else if (launch_tail<T>(s, v, ls, Lv, h->nu1, h->nu2, h->has_ib, h->nr, b[ls], w[ls], h->p<double>(h->cainv)) != 0)
    h->launch_error = true;
  for (int l = ls - 1; l >= 0; --l) {
    launch_prolong_add<T>(s, v[l].N, w[l + 1], w[l], h->walls);
    for (int q = 0; q < h->nu2; ++q) sweep<T>(h, v[l], l, b[l], w[l], r[l]);
  }
}

// Capture the V-cycle of the handle's precision on fixed buffers into a graph.
int capture_vcycle(ibmg_handle* h) {
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
  if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
  std::lock_guard<std::mutex> capture_lock(capture_mutex());
  IBMG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  hipStream_t user = h->stream;
  h->stream = h->cap;
  // the graph starts after precond's input pass, which also clears w0
  if (h->prec == IBMG_FP32) vcycle<float>(h, h->p<float>(h->b0f), h->p<float>(h->w0f), true);
  else vcycle<double>(h, h->p<double>(h->b0g), h->p<double>(h->w0g), true);
  const hipError_t e = hipStreamEndCapture(h->cap, &h->graph);
  h->stream = user;
  if (e != hipSuccess || h->launch_error) return IBMG_EHIP;
  IBMG_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
  h->graph_dt = h->dt;
  return IBMG_OK;
}

// z = M^{-1} r in FP64 at the ABI, dispatching on the V-cycle precision.
// Without event timing the V-cycle runs as a replayed graph.
void precond(ibmg_handle* h, const double* r, double* z) {
  const size_t n0 = h->n0();
  const bool graph = !h->timing && h->cap;
  if (graph && (!h->gexec || h->graph_dt != h->dt)) {
    if (capture_vcycle(h) != IBMG_OK) { h->launch_error = true; return; }
  }
  if (h->prec == IBMG_FP32 && h->fb64) {
    vcycle_fp64(h, r, z);
  } else if (h->prec == IBMG_FP32) {
    yib_for_fp32(h);
    k_vcycle_in<float><<<nblk(n0), 256, 0, h->stream>>>(r, h->p<float>(h->b0f), h->p<float>(h->w0f), n0);
    if (graph) {
      if (hipGraphLaunch(h->gexec, h->stream) != hipSuccess) h->launch_error = true;
    } else {
      vcycle<float>(h, h->p<float>(h->b0f), h->p<float>(h->w0f), true);
    }
    k_convert<float, double><<<nblk(n0), 256, 0, h->stream>>>(h->p<float>(h->w0f), z, n0);
  } else if (graph) {
    k_vcycle_in<double><<<nblk(n0), 256, 0, h->stream>>>(r, h->p<double>(h->b0g), h->p<double>(h->w0g), n0);
    if (hipGraphLaunch(h->gexec, h->stream) != hipSuccess ||
        hipMemcpyAsync(z, h->p<double>(h->w0g), n0 * sizeof(double), hipMemcpyDeviceToDevice, h->stream) !=
            hipSuccess)
      h->launch_error = true;
  } else {
    vcycle<double>(h, r, z);
  }
}

// y = A_0 w (FP64, the outer operator of FGMRES).
void apply0(ibmg_handle* h, const double* w, double* y, const double* b = nullptr) {
  LevelView<double> v = view<double>(h, 0);
  launch_residual<double>(h->stream, v, b, w, y, h->has_ib);
}

// <a, b> into dev[0]
void dot(ibmg_handle* h, const double* a, const double* b, double* dev) {
  launch_multidot(h->stream, a, 0, 1, b, h->n0(), h->p<double>(h->partial), kDotBlocks);
  launch_reduce(h->stream, h->p<double>(h->partial), kDotBlocks, 1, dev, 0);
}

// ---------------------------------------------------------------- setup

}  // namespace

namespace ibmg {

// First half of the per-step setup: points, bins, elastic windows on every
// level and box classes, then the asynchronous read-back of the counts that
// setup_finish checks.  Nothing here waits for the device.
int setup_launch(ibmg_handle* h, double dt, const double* X) {
  if (!h->ws) return IBMG_ENOMEM;
  if (!(dt > 0.0) || !std::isfinite(dt)) return IBMG_EINVAL;
  hipStream_t s = h->stream;
  h->dt = dt;
  h->setup_ok = false;
  h->yib64 = false;   // the elastic-row buffers are cleared below
  const int M = h->M, Lv = h->levels;
  // the explicit method keeps the elastic force on the right-hand side only
  h->has_ib = M > 0 && h->K != 0.0 && h->scheme == IBMG_IMPLICIT;
  int* meta = h->p<int>(h->meta);
  k_fill_i32<<<1, 256, 0, s>>>(meta, 8, 0);
  if (M > 0) {
    if (!X) return IBMG_EINVAL;
    IBMG_HIP(hipMemcpyAsync(h->p<double>(h->X0), X, 2 * (size_t)M * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_fiber_force(s, M, h->p<int>(h->prev_d), h->p<int>(h->next_d), h->K, h->p<double>(h->X0),
                       h->p<double>(h->G));
    launch_weights0(s, M, h->N, h->kind, h->p<double>(h->X0), h->p<int>(h->org), h->p<double>(h->wts));
    launch_box_lists(s, points(h), h->p<int>(h->cnt), h->p<int>(h->start), h->p<int>(h->cursor),
                     h->p<int>(h->list), h->max_list, h->p<int>(h->ltotal), h->p<int>(h->loc), h->p<int>(h->bsum));
  }
  if (h->has_ib) {
    // elastic rows on every level: M_0 from the points, then M_{l+1} = R M_l P
    const double h0 = 1.0 / h->N;
    const double kappa = -dt * h->K / (h0 * h0);
    for (int l = 0; l < Lv; ++l) {
      LevelBufs& B = h->L[l];
      launch_active(s, l, M, B.N, h->p<int>(h->org), l > 0 ? h->p<int>(h->L[l - 1].act) : nullptr,
                    h->p<int>(h->flag), h->p<int>(B.act), h->p<int>(B.rows), h->p<int>(B.nact), B.maxact,
                    h->p<int>(h->loc), h->p<int>(h->bsum));
      if (l == 0)
        launch_windows0(s, points(h), h->p<int>(B.rows), h->p<int>(B.nact), B.maxact, kappa, B.reach,
                        h->p<double>(B.win), meta);
      else
        launch_windows_coarse(s, B.N, h->p<int>(h->L[l - 1].act), h->p<double>(h->L[l - 1].win),
                              h->L[l - 1].maxact, h->L[l - 1].reach, h->p<int>(B.rows), h->p<int>(B.nact),
                              B.maxact, B.reach, h->p<double>(B.win), meta, h->walls ? 1 : 0);
      if (h->prec == IBMG_FP32) {
        const size_t nw = 2 * (size_t)B.maxact * IBMG_WS;
        k_convert<double, float><<<nblk(nw), 256, 0, s>>>(h->p<double>(B.win), h->p<float>(B.winf), nw);
      }
      // elastic rows by face: zero off this step's active rows
      const size_t ny = 2 * (size_t)B.N * B.N;
      k_fill<double><<<nblk(ny), 256, 0, s>>>(h->p<double>(B.yib), ny, 0.0);
      // one-launch four-colour levels: each colour's phase evaluates only
      // the elastic rows of its own boxes
      if (B.crow.bytes)
        launch_colour_rows(s, B.N, h->n, B.nb, h->p<int>(B.rows), h->p<int>(B.nact), B.maxact, h->p<int>(B.crow),
                           h->p<int>(B.ncrow));
    }
  }
  for (int l = 0; l + 1 < Lv; ++l) {
    LevelBufs& B = h->L[l];
    launch_box_classes(s, B.N, h->n, B.nb, h->ncol_l[l], h->has_ib ? h->p<int>(B.act) : nullptr, h->walls ? 1 : 0,
                       h->p<int>(B.boxflag),
                       h->p<int>(B.ib_index), h->p<int>(B.ib_boxes), h->p<int>(B.info));
  }
  // read back counts: boxes with elastic rows per colour, active rows, flags
  h->rb_info.assign(8 * Lv, 0);
  h->rb_nact.assign(2 * Lv, 0);
  h->rb_mt.assign(8, 0);
  h->rb_lt.assign(4, 0);
  for (int l = 0; l + 1 < Lv; ++l)
    IBMG_HIP(hipMemcpyAsync(&h->rb_info[8 * l], h->p<int>(h->L[l].info), 8 * sizeof(int), hipMemcpyDeviceToHost, s));
  if (h->has_ib)
    for (int l = 0; l < Lv; ++l)
      IBMG_HIP(hipMemcpyAsync(&h->rb_nact[2 * l], h->p<int>(h->L[l].nact), 2 * sizeof(int), hipMemcpyDeviceToHost,
                              s));
  IBMG_HIP(hipMemcpyAsync(h->rb_mt.data(), meta, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
  if (M > 0) IBMG_HIP(hipMemcpyAsync(h->rb_lt.data(), h->p<int>(h->ltotal), sizeof(int), hipMemcpyDeviceToHost, s));
  return IBMG_OK;
}

// Second half, after the stream has reached the read-back: capacity and
// window checks, box inverses, coarsest system.  Launches only.
int setup_finish(ibmg_handle* h) {
  hipStream_t s = h->stream;
  const int M = h->M, Lv = h->levels;
  const std::vector<int>&info = h->rb_info, &nact = h->rb_nact, &mt = h->rb_mt, &lt = h->rb_lt;
  if (M > 0 && lt[0] > h->max_list) return IBMG_ENOMEM;
  for (int l = 0; l < Lv && h->has_ib; ++l) {
    if (nact[2 * l] > h->L[l].maxact || nact[2 * l + 1] > h->L[l].maxact) return IBMG_ENOMEM;
    // launch size of the elastic-row passes: grows with the active set (a
    // quarter of headroom), and a V-cycle graph captured with a smaller one
    // is captured again
    const int need = std::max(nact[2 * l], nact[2 * l + 1]);
    if (need > h->L[l].rowhint) {
      h->L[l].rowhint = std::min(h->L[l].maxact, need + need / 4 + 64);
      h->graph_dt = -1.0;
    }
  }
  if (mt[0] != 0) return IBMG_ESHAPE;   // an elastic coupling reaches beyond the coefficient window
  // box inverses of all levels in one launch (the levels are independent)
  BoxFactorLevels F{};
  F.nl = Lv - 1;
  int nfb = 0;
  for (int l = 0; l + 1 < Lv; ++l) {
    for (int c = 0; c < 5; ++c) h->n_ib[l][c] = h->own_boxes() ? info[8 * l + c] : 0;
    if (h->n_ib[l][4] > h->L[l].max_ib) return IBMG_ENOMEM;
    F.v[l] = view<double>(h, l);
    F.ib_boxes[l] = h->p<int>(h->L[l].ib_boxes);
    F.ainv_plain[l] = h->p<double>(h->L[l].ainv_plain);
    F.ainv_plain_f[l] = h->p<float>(h->L[l].ainv_plain_f);
    F.ainv_ib[l] = h->p<double>(h->L[l].ainv_ib);
    F.first[l] = nfb;
    nfb += 1 + h->n_ib[l][4];
  }
  F.first[F.nl] = nfb;
  launch_box_factor(s, F);
  {
    LevelView<double> v = view<double>(h, Lv - 1);
    launch_coarse_assemble(s, v, h->p<double>(h->aug), h->nr);
    if (coarse_factor(s, h->p<double>(h->aug), h->nr, h->p<double>(h->cm), h->p<int>(h->cpiv), nullptr,
                      h->p<int>(h->crowpos), h->p<int>(h->cused), h->p<double>(h->cY), h->p<double>(h->cainv)) != 0)
      return IBMG_EHIP;
  }
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

}  // namespace ibmg

namespace {

int do_setup(ibmg_handle* h, double dt, const double* X) {
  int rc = setup_launch(h, dt, X);
  if (rc) return rc;
  IBMG_HIP(hipStreamSynchronize(h->stream));
  rc = setup_finish(h);
  if (rc) return rc;
  IBMG_HIP(hipStreamSynchronize(h->stream));
  h->setup_ok = true;
  return IBMG_OK;
}

// ---------------------------------------------------------------- FGMRES

int do_solve_impl(ibmg_handle* h, const double* b, double* x, ibmg_stats* st) {
  hipStream_t s = h->stream;
  const size_t n0 = h->n0();
  const int m = h->mb, ldh = m + 1, cap = h->maxit;
  double* V = h->p<double>(h->V);
  double* Z = h->p<double>(h->Z);
  double* H = h->p<double>(h->H);
  double* g = h->p<double>(h->g);
  double* scal = h->p<double>(h->scal);
  double* partial = h->p<double>(h->partial);
  double* hc = h->p<double>(h->hc);
  double* cs = h->p<double>(h->cs);
  double* sn = h->p<double>(h->sn);
  const bool dcgs2 = h->orth == IBMG_ORTH_DCGS2;
  double hs[4];
  h->ev_used = 0;
  dot(h, b, b, scal);
  int rc = read_doubles(h, scal, hs, 1);
  if (rc) return rc;
  const double bnorm = std::sqrt(hs[0]);
  if (!std::isfinite(bnorm)) return IBMG_ENONFINITE;
  st->bnorm = bnorm;
  st->iters = 0;
  st->converged = 0;
  st->fallback = 0;
  h->fb64 = false;
  std::vector<double> hist;   // Arnoldi estimate after each iteration
  st->rel_resid_est = 0;
  st->rel_resid_true = 0;
  if (bnorm == 0.0) {
    k_fill<double><<<nblk(n0), 256, 0, s>>>(x, n0, 0.0);
    st->converged = 1;
    return sync(h);
  }
  const double target = h->rtol * bnorm;
  int total = 0;
  double est = INFINITY;
  // Each cycle starts from the true residual of the current iterate.  The
  // iterate with the smallest true residual so far is kept, and a solve that
  // stops unconverged returns it (a cycle can end worse than it started when
  // its basis was built with a stalled FP32 V-cycle).
  double best = INFINITY;
  double* xbest = h->p<double>(h->xbest);
  for (;;) {
    apply0(h, x, V, b);            // V[0] = b - A x
    dot(h, V, V, scal);
    if ((rc = read_doubles(h, scal, hs, 1))) return rc;
    const double beta = std::sqrt(hs[0]);
    if (!std::isfinite(beta)) return IBMG_ENONFINITE;
    st->rel_resid_true = beta / bnorm;
    if (beta <= target) { st->converged = 1; break; }
    if (beta < best) {
      best = beta;
      if (total < cap) IBMG_HIP(hipMemcpyAsync(xbest, x, n0 * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (total >= cap) {
      if (beta > best) {           // give back the best iterate
        IBMG_HIP(hipMemcpyAsync(x, xbest, n0 * sizeof(double), hipMemcpyDeviceToDevice, s));
        st->rel_resid_true = best / bnorm;
      }
      break;
    }
    launch_scale(s, V, V, n0, scal);
    k_fill<double><<<nblk(m + 2), 256, 0, s>>>(g, m + 2, 0.0);
    IBMG_HIP(hipMemcpyAsync(g, &beta, sizeof(double), hipMemcpyHostToDevice, s));
    int k = 0;
    // Iteration j: preconditioner, operator, classical Gram-Schmidt twice,
    // H(j+1, j) and the Givens step; its flags land in pinned slot j & 1 and
    // an event marks them.
    // Delayed form: V[j] holds u_j until iteration j completes it into v_j
    // (and completes column j - 1); column k - 1 of the last iteration is
    // completed after the loop unless a later iteration was enqueued.
    int enq_max = -1;
    auto enqueue = [&](int j) -> int {
      double* vj = V + (size_t)j * n0;
      double* vn = V + (size_t)(j + 1) * n0;
      double* zj = Z + (size_t)j * n0;
      double* colj = H + (size_t)j * ldh;
      enq_max = j;
      precond(h, vj, zj);
      if (h->launch_error) return IBMG_EHIP;
      apply0(h, zj, vn);
      if (dcgs2) {
        launch_multidot2(s, V, n0, j + 1, vj, vn, n0, partial, kDotBlocks);
        launch_reduce(s, partial, kDotBlocks, 2 * (j + 1), hc, 0);
        launch_dcgs2_coef(s, hc, hc + (j + 1), j - 1, H, ldh, cs, sn, g, scal + 2);
        launch_dcgs2_update(s, V, n0, j, hc, hc + (j + 1), scal + 2, n0, partial);
        launch_reduce2(s, partial, (int)nblk(n0), colj + j + 1, scal + 1);
        launch_scale_tentative(s, vn, n0, scal + 1, H, ldh, g, cs, sn, j, h->flags_d + 4 * (j & 1), target);
        IBMG_HIP(hipEventRecord(h->flag_ev[j & 1], s));
        return IBMG_OK;
      }
      launch_multidot(s, V, n0, j + 1, vn, n0, partial, kDotBlocks);
      launch_reduce(s, partial, kDotBlocks, j + 1, colj, 0);
      launch_update_acc(s, V, n0, j + 1, colj, vn, n0, nullptr);
      launch_multidot(s, V, n0, j + 1, vn, n0, partial, kDotBlocks);
      launch_reduce(s, partial, kDotBlocks, j + 1, hc, 0);
      launch_update_acc(s, V, n0, j + 1, hc, vn, n0, colj);
      launch_multidot(s, vn, 0, 1, vn, n0, partial, kDotBlocks);
      launch_reduce2(s, partial, kDotBlocks, colj + j + 1, scal + 1);
      launch_scale_givens(s, vn, n0, scal + 1, H, ldh, g, h->p<double>(h->cs), h->p<double>(h->sn), j,
                          h->flags_d + 4 * (j & 1), target);
      IBMG_HIP(hipEventRecord(h->flag_ev[j & 1], s));
      return IBMG_OK;
    };
    // Iteration j + 1 is enqueued before iteration j's flags are read, so the
    // device does not wait for the host's decision.  If the cycle stops at j,
    // iteration j + 1 has written only state that the update below does not
    // read (basis vector j + 2, preconditioned vector j + 1, column j + 1 of
    // H, g[j + 1] and g[j + 2], rotation j + 1); the iterates are the same as
    // without the lookahead.  Off while phases are timed.
    const bool lookahead = !h->timing;
    int j = 0;
    bool queued = false;   // iteration j is enqueued
    if (j < m && total < cap) {
      if ((rc = enqueue(0))) return rc;
      queued = true;
    }
    while (queued) {
      const bool ahead = lookahead && j + 1 < m && total + 1 < cap;
      if (ahead && (rc = enqueue(j + 1))) return rc;
      IBMG_HIP(hipEventSynchronize(h->flag_ev[j & 1]));
      for (int q = 0; q < 3; ++q) hs[q] = reinterpret_cast<volatile double*>(h->flags_h)[4 * (j & 1) + q];
      ++total;
      k = j + 1;
      est = hs[0] / bnorm;
      if (hs[2] != 0.0) return IBMG_ENONFINITE;
      hist.push_back(est);
      const int nh = (int)hist.size();
      if (h->prec == IBMG_FP32 && !h->fb64 && nh > kFallbackWindow && est > 0.9 * hist[nh - 1 - kFallbackWindow]) {
        h->fb64 = true;   // FP32 V-cycle stalled: restart from the current iterate with the FP64 one
        st->fallback = 1;
        break;
      }
      if (hs[1] != 0.0) break;
      ++j;
      if (!ahead) {
        queued = j < m && total < cap;
        if (queued && (rc = enqueue(j))) return rc;
      }
    }
    if (dcgs2 && k > 0 && enq_max < k) {   // complete column k - 1 (second projection of u_k)
      const int c = k - 1;
      launch_multidot(s, V, n0, c + 2, V + (size_t)(c + 1) * n0, n0, partial, kDotBlocks);
      launch_reduce(s, partial, kDotBlocks, c + 2, hc, 0);
      launch_dcgs2_coef(s, hc, nullptr, c, H, ldh, cs, sn, g, scal + 2);
    }
    launch_backsolve(s, H, ldh, g, k, h->p<double>(h->y));
    launch_update(s, Z, n0, k, h->p<double>(h->y), x, n0, 1.0);
  }
  st->iters = total;
  st->rel_resid_est = std::isfinite(est) ? est : st->rel_resid_true;
  // phase timings
  if (h->timing && h->ev_used > 0) {
    IBMG_HIP(hipStreamSynchronize(s));
    for (int q = 0; q + 1 < h->ev_used; q += 2) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, h->ev[q], h->ev[q + 1]) == hipSuccess) {
        h->t_total_ms += ms;
        h->t_bytes += h->ev_bytes[q / 2];
        h->t_launches += 1;
      }
    }
  }
  return st->converged ? IBMG_OK : IBMG_NOT_CONVERGED;
}

// Multigrid as the solver (Sec. 5.1): w <- w + MGV(0, b - A w), the V-cycle
// of the handle's precision applied to the FP64 residual, until
// ||b - A w|| <= rtol ||b|| or maxit V-cycles.  A diverging iteration (the
// paper's MG alone at high stiffness) stops once the residual has grown by
// 1e12 and reports IBMG_NOT_CONVERGED.
int do_solve_mg(ibmg_handle* h, const double* b, double* x, ibmg_stats* st) {
  hipStream_t s = h->stream;
  const size_t n0 = h->n0();
  double* r = h->p<double>(h->V);
  double* z = h->p<double>(h->Z);
  double* scal = h->p<double>(h->scal);
  double hs[1];
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
    k_fill<double><<<nblk(n0), 256, 0, s>>>(x, n0, 0.0);
    st->converged = 1;
    return sync(h);
  }
  const double target = h->rtol * bnorm;
  for (;;) {
    apply0(h, x, r, b);   // r = b - A w
    dot(h, r, r, scal);
    if ((rc = read_doubles(h, scal, hs, 1))) return rc;
    const double beta = std::sqrt(hs[0]);
    if (!std::isfinite(beta)) return IBMG_ENONFINITE;
    st->rel_resid_true = st->rel_resid_est = beta / bnorm;
    if (beta <= target) { st->converged = 1; break; }
    if (st->iters >= h->maxit || beta > 1e12 * bnorm) break;
    precond(h, r, z);
    if (h->launch_error) return IBMG_EHIP;
    k_lincomb<<<nblk(n0), 256, 0, s>>>(x, x, z, 1.0, nullptr, 0.0, n0);
    ++st->iters;
  }
  return st->converged ? IBMG_OK : IBMG_NOT_CONVERGED;
}

// The FP64 fallback belongs to one solve: whatever way the solve ends, later
// V-cycles (the next solve, ibmg_vcycle) run in the handle's precision.
int do_solve(ibmg_handle* h, const double* b, double* x, ibmg_stats* st) {
  const int rc = h->solver == IBMG_SOLVER_MG ? do_solve_mg(h, b, x, st) : do_solve_impl(h, b, x, st);
  h->fb64 = false;
  return rc;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool ready(const ibmg_handle* h) { return h && h->ws; }

}  // namespace

namespace ibmg {

int bind(ibmg_handle* h, void* dev, size_t bytes, bool own_capture_stream) {
  if (!h || !dev) return IBMG_EINVAL;
  char* base = (char*)(((uintptr_t)dev + 255) & ~(uintptr_t)255);
  if (bytes < h->need || (size_t)(base - (char*)dev) + h->need - 256 > bytes) return IBMG_ENOMEM;
  h->ws = base;
  h->ws_bytes = bytes;
  h->setup_ok = false;
  h->graph_dt = -1.0;
  if (own_capture_stream && !h->cap) IBMG_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  if (!h->flags_h) {
    // the per-iteration flags of FGMRES go straight to host memory (two
    // slots, for the iteration being read and the one enqueued after it): no
    // copy is enqueued between the Givens step and the host's decision
    IBMG_HIP(hipHostMalloc((void**)&h->flags_h, 8 * sizeof(double), hipHostMallocDefault));
    IBMG_HIP(hipHostGetDevicePointer((void**)&h->flags_d, h->flags_h, 0));
    for (auto& e : h->flag_ev) IBMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // dynamic LDS of the V-cycle tail (levels of at most kSmallLevel cells per side)
  if (prepare_tail(tail_lds(h, sizeof(double))) != 0) return IBMG_EHIP;
  if (h->M > 0) {
    IBMG_HIP(hipMemcpyAsync(h->p<int>(h->prev_d), h->prev.data(), h->M * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
    IBMG_HIP(hipMemcpyAsync(h->p<int>(h->next_d), h->next.data(), h->M * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
    IBMG_HIP(hipStreamSynchronize(h->stream));
  }
  return IBMG_OK;
}

// Zero the elastic-row buffers of every level (they must be zero off the
// active rows, in whichever precision the next V-cycle reads them).
void clear_yib(ibmg_handle* h) {
  for (int l = 0; l < h->levels; ++l) {
    const size_t ny = 2 * (size_t)h->L[l].N * h->L[l].N;
    k_fill<double><<<nblk(ny), 256, 0, h->stream>>>(h->p<double>(h->L[l].yib), ny, 0.0);
  }
}

void vcycle_fp64(ibmg_handle* h, const double* r, double* z) {
  // on an FP32 handle the elastic-row buffers hold FP32 values: read as FP64
  // off the active rows they would not be zero, so clear them first (and once
  // more before the next FP32 V-cycle, which would read these FP64 values)
  if (h->prec == IBMG_FP32 && h->has_ib) {
    if (!h->yib64) clear_yib(h);
    h->yib64 = true;
  }
  vcycle<double>(h, r, z);
}

// Before an FP32 V-cycle or smoothing pass: undo what an FP64 fallback
// V-cycle left in the elastic-row buffers.
void yib_for_fp32(ibmg_handle* h) {
  if (h->prec == IBMG_FP32 && h->has_ib && h->yib64) {
    clear_yib(h);
    h->yib64 = false;
  }
}

// Right-hand side (a4) into bvec and the initial iterate into xvec.
int step_begin(ibmg_handle* h, double dt, const double* u, const double* v, const double* p, const double* gu,
               const double* gv) {
  hipStream_t s = h->stream;
  const size_t NN = (size_t)h->N * h->N, n0 = h->n0();
  double* b = h->p<double>(h->bvec);
  double* x = h->p<double>(h->xvec);
  launch_rhs(s, points(h), h->rho / dt, (double)h->N * h->N, u, v, gu, gv, h->M > 0 ? h->p<double>(h->G) : nullptr,
             b, h->walls ? 1 : 0, h->mu);
  if (h->guess == IBMG_GUESS_PREV) {
    IBMG_HIP(hipMemcpyAsync(x, u, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(x + NN, v, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(x + 2 * NN, p, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    k_fill<double><<<nblk(n0), 256, 0, s>>>(x, n0, 0.0);
  }
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

// Zero-mean pressure, then move the structure with the lagged S^n (a14) and
// copy the new state out.  Launches only.
int step_end(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X) {
  hipStream_t s = h->stream;
  const size_t NN = (size_t)h->N * h->N;
  double* x = h->p<double>(h->xvec);
  double* part = h->p<double>(h->partial);
  double* scal = h->p<double>(h->scal);
  launch_sum(s, x + 2 * NN, NN, part, kDotBlocks);
  launch_reduce(s, part, kDotBlocks, 1, scal, 0);
  launch_mean_shift(s, x + 2 * NN, NN, scal);
  if (h->M > 0) launch_interp(s, points(h), x, x + NN, h->p<double>(h->U), h->p<double>(h->X0), dt);
  IBMG_HIP(hipMemcpyAsync(u, x, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
  IBMG_HIP(hipMemcpyAsync(v, x + NN, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
  IBMG_HIP(hipMemcpyAsync(p, x + 2 * NN, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h->M > 0)
    IBMG_HIP(hipMemcpyAsync(X, h->p<double>(h->X0), 2 * (size_t)h->M * sizeof(double), hipMemcpyDeviceToDevice, s));
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

}  // namespace ibmg

// ====================================================================== C ABI
extern "C" {

const char* ibmg_status_string(int s) {
  switch (s) {
    case IBMG_OK: return "ok";
    case IBMG_NOT_CONVERGED: return "not converged (iteration cap)";
    case IBMG_EINVAL: return "invalid argument";
    case IBMG_ESHAPE: return "unsupported shape (N, levels or box size)";
    case IBMG_EHIP: return "HIP runtime error";
    case IBMG_ENOMEM: return "workspace too small or not bound";
    case IBMG_ENONFINITE: return "non-finite value";
    case IBMG_ESTATE: return "call order violated (setup missing)";
    default: return "unknown status";
  }
}

int ibmg_create(ibmg_handle** out, const ibmg_problem* pr, const ibmg_opts* op, void* stream) {
  if (!out || !pr || !op) return IBMG_EINVAL;
  *out = nullptr;
  const int N = pr->N;
  if (N < 4 || (N & (N - 1)) != 0) return IBMG_ESHAPE;
  if (pr->domain != IBMG_PERIODIC && pr->domain != IBMG_CAVITY) return IBMG_EINVAL;
  const bool cavity = pr->domain == IBMG_CAVITY;
  // periodic: rho > 0 (the steady periodic problem leaves the velocity's mean free)
  if (!(pr->rho > 0 || (cavity && pr->rho == 0)) || !(pr->mu > 0) || !std::isfinite(pr->K) || pr->K < 0)
    return IBMG_EINVAL;
  if (cavity && op->tail_max != 1) return IBMG_EINVAL;
  if (pr->delta != IBMG_DELTA_IB4 && pr->delta != IBMG_DELTA_COS4) return IBMG_EINVAL;
  if (op->box != 1 && op->box != 2 && op->box != 4 && op->box != 8) return IBMG_ESHAPE;
  if (op->levels < 1 || op->levels > IBMG_MAX_LEVELS) return IBMG_ESHAPE;
  const int Nc = N >> (op->levels - 1);
  if (Nc < 4 || Nc > 16) return IBMG_ESHAPE;
  for (int l = 0; l + 1 < op->levels; ++l) {
    const int Nl = N >> l;
    if (Nl < 4 || Nl < 2 * op->box) return IBMG_ESHAPE;
  }
  if (op->nu1 < 0 || op->nu2 < 0 || !(op->rtol > 0)) return IBMG_EINVAL;
  if (op->restart < 0 || op->restart > kMaxBasis || op->maxit < 1 ||
      op->maxit > (op->restart == 0 ? kMaxBasis : kMaxIters))
    return IBMG_EINVAL;
  if (op->vcycle_prec != IBMG_FP64 && op->vcycle_prec != IBMG_FP32) return IBMG_EINVAL;
  if (op->guess != IBMG_GUESS_ZERO && op->guess != IBMG_GUESS_PREV) return IBMG_EINVAL;
  if (op->colours != 2 && op->colours != 4) return IBMG_EINVAL;
  if (op->colours_from < 0 || op->colours_from > op->levels) return IBMG_EINVAL;
  if (op->scheme != IBMG_IMPLICIT && op->scheme != IBMG_EXPLICIT) return IBMG_EINVAL;
  if (op->solver != IBMG_SOLVER_FGMRES && op->solver != IBMG_SOLVER_MG) return IBMG_EINVAL;
  if (!(op->omega >= 0.0 && op->omega <= 1.0)) return IBMG_EINVAL;
  if (op->orth != IBMG_ORTH_CGS2 && op->orth != IBMG_ORTH_DCGS2) return IBMG_EINVAL;
  if (op->tail_max != 0 && (op->tail_max < 1 || op->tail_max > kSmallLevel || (op->tail_max & (op->tail_max - 1))))
    return IBMG_EINVAL;
  if (pr->n_points < 0 || pr->n_fibers < 0) return IBMG_EINVAL;
  if (pr->n_points > 0 && (!pr->fiber_offsets || pr->n_fibers < 1)) return IBMG_EINVAL;
  ibmg_handle* h = new (std::nothrow) ibmg_handle();
  if (!h) return IBMG_EINVAL;
  h->N = N; h->M = pr->n_points; h->nfib = pr->n_fibers; h->kind = pr->delta;
  h->rho = pr->rho; h->mu = pr->mu; h->K = pr->K;
  h->walls = cavity;
  h->levels = op->levels; h->n = op->box; h->nu1 = op->nu1; h->nu2 = op->nu2; h->maxit = op->maxit;
  h->mb = op->restart == 0 ? op->maxit : std::min(op->restart, op->maxit);
  h->scheme = op->scheme;
  h->solver = op->solver;
  h->omega = op->omega == 0.0 ? 1.0 : op->omega;
  h->orth = op->orth;
  h->rtol = op->rtol; h->prec = op->vcycle_prec; h->guess = op->guess; h->ncol = op->colours;
  for (int l = 0; l < IBMG_MAX_LEVELS; ++l) h->ncol_l[l] = (op->colours_from > 0 && l >= op->colours_from) ? 2 : op->colours;
  h->tail_max = op->tail_max ? op->tail_max : kSmallLevel;
  h->stream = (hipStream_t)stream;
  h->prev.assign(h->M, 0);
  h->next.assign(h->M, 0);
  if (h->M > 0) {
    const int* o = pr->fiber_offsets;
    if (o[0] != 0 || o[pr->n_fibers] != h->M) { delete h; return IBMG_EINVAL; }
    for (int f = 0; f < pr->n_fibers; ++f)
      if (o[f + 1] < o[f] || o[f + 1] > h->M) { delete h; return IBMG_EINVAL; }
    for (int f = 0; f < pr->n_fibers; ++f) {
      const int a = o[f], b = o[f + 1];
      const int nf = b - a;
      for (int k = a; k < b; ++k) {
        h->prev[k] = a + (k - a - 1 + nf) % nf;
        h->next[k] = a + (k - a + 1) % nf;
      }
    }
  }
  layout(h);
  *out = h;
  return IBMG_OK;
}

int ibmg_workspace_bytes(const ibmg_handle* h, size_t* bytes) {
  if (!h || !bytes) return IBMG_EINVAL;
  *bytes = h->need;
  return IBMG_OK;
}

int ibmg_bind_workspace(ibmg_handle* h, void* dev, size_t bytes) {
  return bind(h, dev, bytes, true);
}

int ibmg_destroy(ibmg_handle* h) {
  if (!h) return IBMG_EINVAL;
  for (auto e : h->ev) (void)hipEventDestroy(e);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->flags_h) (void)hipHostFree(h->flags_h);
  for (auto e : h->flag_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
  return IBMG_OK;
}

int ibmg_set_timing(ibmg_handle* h, int on) {
  if (!h) return IBMG_EINVAL;
  h->timing = on != 0;
  if (h->timing && h->ev.empty()) {
    h->ev.resize(2 * kMaxTimed);
    for (auto& e : h->ev) IBMG_HIP(hipEventCreate(&e));
    h->ev_bytes.assign(kMaxTimed, 0.0);
  }
  h->t_total_ms = 0;
  h->t_bytes = 0;
  h->t_launches = 0;
  return IBMG_OK;
}

int ibmg_phase_timing(ibmg_handle* h, double* total_ms, int64_t* launches, double* bytes) {
  if (!h) return IBMG_EINVAL;
  if (total_ms) *total_ms = h->t_total_ms;
  if (launches) *launches = h->t_launches;
  if (bytes) *bytes = h->t_bytes;
  return IBMG_OK;
}

}  // extern "C"

namespace {

template <typename T>
int box_bench(ibmg_handle* h, int level, int colour, int reps, double* avg_us, double* bytes) {
  LevelView<T> v = view<T>(h, level);
  T* w = (level == 0 && h->prec == IBMG_FP64) ? h->p<T>(h->w0g) : h->p<T>(h->L[level].w);
  T* r = h->p<T>(h->L[level].r);
  // the launches are captured into a graph and replayed between the events,
  // so that host launch overhead does not leave the GPU idle between them
  if (!h->cap) return IBMG_ESTATE;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  std::lock_guard<std::mutex> capture_lock(capture_mutex());
  IBMG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  // the box launch the V-cycle makes: on four-colour levels the one that forms
  // its own Stokes residuals from b (the elastic rows as last evaluated)
  const bool fused = phase_fusable(v.ncol, v.n);
  const T* b = (level == 0 && h->prec == IBMG_FP64) ? h->p<T>(h->b0g) : h->p<T>(h->L[level].b);
  for (int q = 0; q < reps; ++q) {
    if (fused) launch_phase_fused<T>(h->cap, v, b, w, colour, h->own_boxes(), false);
    else launch_box<T>(h->cap, v, r, w, colour, h->own_boxes());
  }
  IBMG_HIP(hipStreamEndCapture(h->cap, &g));
  if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return IBMG_EHIP;
  }
  hipEvent_t e0, e1;
  IBMG_HIP(hipEventCreate(&e0));
  IBMG_HIP(hipEventCreate(&e1));
  IBMG_HIP(hipGraphLaunch(ge, h->stream));   // warm-up replay
  IBMG_HIP(hipEventRecord(e0, h->stream));
  IBMG_HIP(hipGraphLaunch(ge, h->stream));
  IBMG_HIP(hipEventRecord(e1, h->stream));
  IBMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return IBMG_EHIP;
  if (avg_us) *avg_us = 1e3 * (double)ms / reps;
  if (bytes) {
    // per box: read the residual (or b) and the iterate, write the iterate at
    // every unknown; a fused launch also reads the iterate on the box's
    // one-cell halo (10 n + 4 values: the x and y neighbours of its u and v
    // faces and the pressures left and below)
    const double boxes = colour_count(v.ncol, v.nb);
    const double per_box = v.ndof * 3.0 + (fused ? 10.0 * v.n + 4.0 : 0.0);
    double by = boxes * per_box * sizeof(T) + (double)v.ndof * v.ndof * sizeof(T);
    if (h->own_boxes()) by += (double)h->n_ib[level][colour] * v.ndof * v.ndof * sizeof(double);
    *bytes = by;
  }
  return IBMG_OK;
}

// Graph-replayed timing of one hot-path kernel (see ibmg_kernel_bench):
// `reps` launches captured on the capture stream, replayed once to warm up,
// then once between two HIP events on the handle's stream.
template <typename F>
int replay_time(ibmg_handle* h, int reps, F launch, double* avg_us) {
  if (!h->cap) return IBMG_ESTATE;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  std::lock_guard<std::mutex> capture_lock(capture_mutex());
  IBMG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  for (int q = 0; q < reps; ++q) launch(h->cap);
  IBMG_HIP(hipStreamEndCapture(h->cap, &g));
  if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return IBMG_EHIP;
  }
  hipEvent_t e0, e1;
  IBMG_HIP(hipEventCreate(&e0));
  IBMG_HIP(hipEventCreate(&e1));
  IBMG_HIP(hipGraphLaunch(ge, h->stream));
  IBMG_HIP(hipEventRecord(e0, h->stream));
  IBMG_HIP(hipGraphLaunch(ge, h->stream));
  IBMG_HIP(hipEventRecord(e1, h->stream));
  IBMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return IBMG_EHIP;
  *avg_us = 1e3 * (double)ms / reps;
  return IBMG_OK;
}

// The fused residual pass of a colour phase on level `level` (k_res_ib), in
// the handle's V-cycle precision, on the level's V-cycle vectors.
template <typename T>
int res_bench(ibmg_handle* h, int level, int reps, double* avg_us, double* bytes) {
  LevelView<T> v = view<T>(h, level);
  T* w = (level == 0 && h->prec == IBMG_FP64) ? h->p<T>(h->w0g) : h->p<T>(h->L[level].w);
  const T* b = (level == 0 && h->prec == IBMG_FP64) ? h->p<T>(h->b0g) : h->p<T>(h->L[level].b);
  T* r = h->p<T>(h->L[level].r);
  const int rc = replay_time(h, reps, [&](hipStream_t s) { launch_res<T>(s, v, b, w, r, h->has_ib); }, avg_us);
  if (rc) return rc;
  // read w and b, write r on every unknown; per active elastic row its window
  // (121 coefficients) and the window's iterate values, and the row's result
  const double n3 = 3.0 * v.N * v.N;
  double by = 3.0 * n3 * sizeof(T);
  if (h->has_ib) {
    const double rows = (double)h->rb_nact[2 * level] + h->rb_nact[2 * level + 1];
    by += rows * (IBMG_WS * sizeof(T) + sizeof(int) + sizeof(T));
  }
  *bytes = by;
  return IBMG_OK;
}

}  // namespace

extern "C" {

int ibmg_kernel_bench(ibmg_handle* h, int kernel, int level, int arg, int reps, double* avg_us, double* bytes) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (reps < 1 || !avg_us || !bytes) return IBMG_EINVAL;
  const size_t n0 = h->n0();
  double* V = h->p<double>(h->V);
  switch (kernel) {
    case IBMG_KERNEL_BOX:
      return ibmg_box_bench(h, level, arg, reps, avg_us, bytes);
    case IBMG_KERNEL_RES:
      if (level < 0 || level + 1 >= h->levels) return IBMG_EINVAL;
      return h->prec == IBMG_FP32 ? res_bench<float>(h, level, reps, avg_us, bytes)
                                  : res_bench<double>(h, level, reps, avg_us, bytes);
    case IBMG_KERNEL_MULTIDOT: {
      // <V_i, v_arg> for i < arg over the FGMRES basis (one Gram-Schmidt pass)
      if (arg < 1 || arg > h->mb) return IBMG_EINVAL;
      double* part = h->p<double>(h->partial);
      const int rc = replay_time(
          h, reps, [&](hipStream_t s) { launch_multidot(s, V, n0, arg, V + (size_t)arg * n0, n0, part, kDotBlocks); },
          avg_us);
      // the arg basis vectors and the new vector once (the kernel reads the
      // new vector again for each group of eight basis vectors; those reads
      // hit L2 and are not counted)
      *bytes = ((double)arg + 1.0) * n0 * sizeof(double);
      return rc;
    }
    case IBMG_KERNEL_UPDATE: {
      // v_arg -= sum_{i < arg} c_i V_i with c = the Hessenberg column (values
      // as left by the last solve; the timing does not depend on them)
      if (arg < 1 || arg > h->mb) return IBMG_EINVAL;
      const double* c = h->p<double>(h->hc);
      const int rc = replay_time(
          h, reps, [&](hipStream_t s) { launch_update_acc(s, V, n0, arg, c, V + (size_t)arg * n0, n0, nullptr); },
          avg_us);
      // the arg basis vectors, read and write the updated vector
      *bytes = ((double)arg + 2.0) * n0 * sizeof(double);
      return rc;
    }
    case IBMG_KERNEL_DOT2: {
      // the delayed form's product pass: V[0 .. arg] against V[arg] and V[arg + 1]
      if (arg < 1 || arg + 1 > h->mb) return IBMG_EINVAL;
      double* part = h->p<double>(h->partial);
      const int rc = replay_time(
          h, reps,
          [&](hipStream_t s) {
            launch_multidot2(s, V, n0, arg + 1, V + (size_t)arg * n0, V + (size_t)(arg + 1) * n0, n0, part,
                             kDotBlocks);
          },
          avg_us);
      // the arg + 1 basis vectors and the two vectors once (the kernel reads
      // the two again for each group of sixteen; those reads hit L2 and are
      // not counted: HBM reads measured 1.0 x this at 60 vectors)
      *bytes = ((double)(arg + 1) + 2.0) * n0 * sizeof(double);
      return rc;
    }
    case IBMG_KERNEL_UPDATE2: {
      // the delayed form's update pass with arg vectors, on zero coefficients
      // and 1 / rho = 1 (V unchanged; the timing does not depend on the values)
      if (arg < 1 || arg + 1 > h->mb) return IBMG_EINVAL;
      hipStream_t s0 = h->stream;
      double* c = h->p<double>(h->hc);
      double* coef = h->p<double>(h->scal) + 2;
      k_fill<double><<<nblk(2 * (size_t)arg), 256, 0, s0>>>(c, 2 * (size_t)arg, 0.0);
      k_fill<double><<<1, 256, 0, s0>>>(coef, 1, 1.0);
      k_fill<double><<<1, 256, 0, s0>>>(coef + 1, 1, 0.0);
      double* part = h->p<double>(h->partial);
      const int rc = replay_time(
          h, reps, [&](hipStream_t s) { launch_dcgs2_update(s, V, n0, arg, c, c + arg, coef, n0, part); },
          avg_us);
      // the arg basis vectors, read and write u and w
      *bytes = ((double)arg + 4.0) * n0 * sizeof(double);
      return rc;
    }
    default:
      return IBMG_EINVAL;
  }
}

int ibmg_box_bench(ibmg_handle* h, int level, int colour, int reps, double* avg_us, double* bytes) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (level < 0 || level + 1 >= h->levels || colour < 0 || colour >= h->ncol_l[level] || reps < 1)
    return IBMG_EINVAL;
  return h->prec == IBMG_FP32 ? box_bench<float>(h, level, colour, reps, avg_us, bytes)
                              : box_bench<double>(h, level, colour, reps, avg_us, bytes);
}

int ibmg_setup(ibmg_handle* h, double dt, const double* X) {
  if (!ready(h)) return IBMG_ENOMEM;
  return do_setup(h, dt, X);
}

int ibmg_rhs(ibmg_handle* h, const double* u, const double* v, const double* gu, const double* gv, double* b) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (!b) return IBMG_EINVAL;
  const double inv_h2 = (double)h->N * h->N;
  launch_rhs(h->stream, points(h), h->rho / h->dt, inv_h2, u, v, gu, gv, h->M > 0 ? h->p<double>(h->G) : nullptr, b,
             h->walls ? 1 : 0, h->mu);
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}

int ibmg_solve(ibmg_handle* h, const double* b, double* w, ibmg_stats* out) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (!b || !w) return IBMG_EINVAL;
  ibmg_stats st{};
  const double t0 = now_ms();
  const size_t n0 = h->n0();
  double* x = h->p<double>(h->xvec);
  IBMG_HIP(hipMemcpyAsync(x, w, n0 * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  int rc = do_solve(h, b, x, &st);
  if (rc >= 0) {
    IBMG_HIP(hipMemcpyAsync(w, x, n0 * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    IBMG_HIP(hipStreamSynchronize(h->stream));
  }
  st.t_solve_ms = now_ms() - t0;
  if (out) *out = st;
  return rc;
}

}  // extern "C"

namespace {

// One implicit step; x0 (nullable) is a proposed initial iterate, used only
// when its residual is below that of w^n.
int step_impl(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X, const double* gu,
              const double* gv, const double* x0, ibmg_stats* out, double t_setup_ms = -1.0) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!u || !v || !p || (h->M > 0 && !X)) return IBMG_EINVAL;
  ibmg_stats st{};
  // t_setup_ms >= 0: the caller has set up at (dt, X) already and took that long
  const double t0 = now_ms() - (t_setup_ms >= 0.0 ? t_setup_ms : 0.0);
  int rc = t_setup_ms >= 0.0 ? IBMG_OK : do_setup(h, dt, X);
  if (rc) return rc;
  const double t1 = now_ms();
  if ((rc = step_begin(h, dt, u, v, p, gu, gv))) return rc;
  if (x0) {
    // x = w^n + alpha (x0 - w^n), alpha minimising ||b - A x||: with
    // r = b - A w^n and q = A (x0 - w^n), alpha = <r, q> / <q, q>, so the
    // start is never worse than w^n
    hipStream_t s = h->stream;
    const size_t NN = (size_t)h->N * h->N, n0 = h->n0();
    double* x = h->p<double>(h->xvec);
    double* b = h->p<double>(h->bvec);
    double* V = h->p<double>(h->V);
    double* scal = h->p<double>(h->scal);
    double* d = h->p<double>(h->rvec);
    IBMG_HIP(hipMemcpyAsync(x, u, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(x + NN, v, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(x + 2 * NN, p, NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(d, x0, n0 * sizeof(double), hipMemcpyDeviceToDevice, s));
    k_fill<double><<<1, 64, 0, s>>>(scal + 8, 1, 1.0);
    launch_update(s, x, n0, 1, scal + 8, d, n0, -1.0);   // d = x0 - w^n
    apply0(h, x, V, b);                                 // r
    apply0(h, d, V + n0);                               // q
    dot(h, V, V + n0, scal + 4);
    dot(h, V + n0, V + n0, scal + 5);
    double hs[2];
    if ((rc = read_doubles(h, scal + 4, hs, 2))) return rc;
    const double alpha = (hs[1] > 0.0 && std::isfinite(hs[0]) && std::isfinite(hs[1])) ? hs[0] / hs[1] : 0.0;
    if (alpha != 0.0) {
      IBMG_HIP(hipMemcpyAsync(scal + 9, &alpha, sizeof(double), hipMemcpyHostToDevice, s));
      launch_update(s, d, n0, 1, scal + 9, x, n0, 1.0);
      IBMG_HIP(hipStreamSynchronize(s));   // alpha lives on the host stack
    } else {
      st.guess_rejected = 1;
    }
    st.guess_alpha = alpha;
  }  const int rejected = st.guess_rejected;
  rc = do_solve(h, h->p<double>(h->bvec), h->p<double>(h->xvec), &st);
  st.guess_rejected = rejected;
  const double t2 = now_ms();
  if (rc < 0) return rc;
  const int rc_end = step_end(h, dt, u, v, p, X);
  if (rc_end) return rc_end;
  IBMG_HIP(hipStreamSynchronize(h->stream));
  h->setup_ok = false;   // the operator belongs to X^n
  st.t_setup_ms = t1 - t0;
  st.t_solve_ms = t2 - t1;
  st.t_step_ms = now_ms() - t0;
  if (out) *out = st;
  return rc;
}

}  // namespace

extern "C" {

int ibmg_step(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X, const double* gu,
              const double* gv, ibmg_stats* out) {
  return step_impl(h, dt, u, v, p, X, gu, gv, nullptr, out);
}

int ibmg_step_x0(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X, const double* gu,
                 const double* gv, const double* x0, ibmg_stats* out) {
  if (!x0) return IBMG_EINVAL;
  return step_impl(h, dt, u, v, p, X, gu, gv, x0, out);
}

int ibmg_guess_step(ibmg_handle* h, ibmg_cnn* c, int mode, double dt, double* u, double* v, double* p, double* X,
                    const double* gu, const double* gv, ibmg_stats* out) {
  if (!ready(h)) return IBMG_ENOMEM;
  CnnTraj T;
  if (!c || cnn_traj(c, &T) != IBMG_OK) return IBMG_ENOMEM;
  if (T.N != h->N || T.stream != h->stream) return IBMG_EINVAL;
  if (mode != IBMG_GUESS_RECORD && mode != IBMG_GUESS_EXTRAP && mode != IBMG_GUESS_LEARNED) return IBMG_EINVAL;
  if (!u || !v || !p || (h->M > 0 && !X)) return IBMG_EINVAL;
  hipStream_t s = h->stream;
  const size_t NN = (size_t)h->N * h->N, n3 = 3 * NN;
  const double t0 = now_ms();
  int rc = do_setup(h, dt, X);   // S at X^n: the features use it
  if (rc) return rc;
  // features (u^n, v^n, p^n, S_0 G^n on u and v faces) and w^n
  double* const w_in[3] = {u, v, p};
  for (int k = 0; k < 3; ++k) {
    IBMG_HIP(hipMemcpyAsync(T.feat + k * NN, w_in[k], NN * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipMemcpyAsync(T.wold + k * NN, w_in[k], NN * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  launch_rhs(s, points(h), 0.0, (double)NN, nullptr, nullptr, nullptr, nullptr,
             h->M > 0 ? h->p<double>(h->G) : nullptr, T.feat + 3 * NN);
  const double* x0 = nullptr;
  const int guess = h->guess;
  if (mode == IBMG_GUESS_RECORD) {
    h->guess = IBMG_GUESS_PREV;
  } else {
    // x0 = w^n + dw^{n-1} (+ the network's correction)
    if (mode == IBMG_GUESS_LEARNED) {
      if ((rc = ibmg_cnn_infer(c, T.feat, T.x0)) != IBMG_OK) return rc;
      k_lincomb<<<nblk(n3), 256, 0, s>>>(T.x0, T.wold, T.dprev, 1.0, T.x0, 1.0, n3);
    } else {
      k_lincomb<<<nblk(n3), 256, 0, s>>>(T.x0, T.wold, T.dprev, 1.0, nullptr, 0.0, n3);
    }
    x0 = T.x0;
  }
  rc = step_impl(h, dt, u, v, p, X, gu, gv, x0, out, now_ms() - t0);
  h->guess = guess;
  if (rc < 0) return rc;
  // dw^n = w^{n+1} - w^n; recording: the pair (features, dw^n - dw^{n-1})
  for (int k = 0; k < 3; ++k)
    k_lincomb<<<nblk(NN), 256, 0, s>>>(T.dw + k * NN, w_in[k], T.wold + k * NN, -1.0, nullptr, 0.0, NN);
  if (mode == IBMG_GUESS_RECORD) {
    k_lincomb<<<nblk(n3), 256, 0, s>>>(T.x0, T.dw, T.dprev, -1.0, nullptr, 0.0, n3);
    const int rr = ibmg_cnn_record(c, T.feat, T.x0);
    if (rr != IBMG_OK) return rr;
  }
  IBMG_HIP(hipMemcpyAsync(T.dprev, T.dw, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  IBMG_HIP(hipStreamSynchronize(s));
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------- single operations

namespace {

template <typename T>
int single_op(ibmg_handle* h, int which, int level, const double* a, const double* b, double* out, int sweeps) {
  hipStream_t s = h->stream;
  if (level < 0 || level >= h->levels) return IBMG_EINVAL;
  LevelView<T> v = view<T>(h, level);
  const size_t n3 = 3 * (size_t)v.N * v.N;
  const bool f32 = sizeof(T) == sizeof(float);
  if (f32) yib_for_fp32(h);
  // staging: FP32 handles convert through the level's r and w buffers (level 0: w0f, b0f)
  auto stage = [&](const double* src, const Buf& bf) -> T* {
    T* d = h->p<T>(bf);
    k_convert<double, T><<<nblk(n3), 256, 0, s>>>(src, d, n3);
    return d;
  };
  const Buf& wb = level == 0 ? h->w0f : h->L[level].w;
  const Buf& bb = level == 0 ? h->b0f : h->L[level].b;
  switch (which) {
    case 0: {  // apply
      const T* w = f32 ? stage(a, wb) : (const T*)a;
      T* y = f32 ? h->p<T>(h->L[level].r) : (T*)out;
      launch_residual<T>(s, v, nullptr, w, y, h->has_ib);
      if (f32) k_convert<T, double><<<nblk(n3), 256, 0, s>>>(y, out, n3);
      break;
    }
    case 1: {  // residual r = b - A w
      const T* w = f32 ? stage(a, wb) : (const T*)a;
      const T* bv = f32 ? stage(b, bb) : (const T*)b;
      T* y = f32 ? h->p<T>(h->L[level].r) : (T*)out;
      launch_residual<T>(s, v, bv, w, y, h->has_ib);
      if (f32) k_convert<T, double><<<nblk(n3), 256, 0, s>>>(y, out, n3);
      break;
    }
    case 2: {  // smooth in place on out, rhs b
      if (level >= h->levels - 1) return IBMG_EINVAL;
      T* w = f32 ? stage(out, wb) : (T*)out;
      const T* bv = f32 ? stage(b, bb) : (const T*)b;
      T* rr = h->p<T>(h->L[level].r);
      for (int q = 0; q < sweeps; ++q) sweep<T>(h, v, level, bv, w, rr);
      if (f32) k_convert<T, double><<<nblk(n3), 256, 0, s>>>(w, out, n3);
      break;
    }
    case 3: {  // restrict a (level) -> out (level+1)
      if (level >= h->levels - 1) return IBMG_EINVAL;
      if (f32) {
        T* f = stage(a, h->L[level].r);
        T* c = h->p<T>(h->L[level + 1].b);
        launch_restrict<T>(s, v.N, f, c, (T*)nullptr, nullptr, h->walls);
        const size_t nc3 = n3 / 4;
        k_convert<T, double><<<nblk(nc3), 256, 0, s>>>(c, out, nc3);
      } else {
        launch_restrict<T>(s, v.N, (const T*)a, (T*)out, (T*)nullptr, nullptr, h->walls);
      }
      break;
    }
    case 4: {  // out (level) += P a (level+1)
      if (level >= h->levels - 1) return IBMG_EINVAL;
      if (f32) {
        const size_t nc3 = n3 / 4;
        T* c = h->p<T>(h->L[level + 1].w);
        k_convert<double, T><<<nblk(nc3), 256, 0, s>>>(a, c, nc3);
        T* f = stage(out, wb);
        launch_prolong_add<T>(s, v.N, c, f, h->walls);
        k_convert<T, double><<<nblk(n3), 256, 0, s>>>(f, out, n3);
      } else {
        launch_prolong_add<T>(s, v.N, (const T*)a, (T*)out, h->walls);
      }
      break;
    }
    case 5: {  // coarsest solve
      const int lc = h->levels - 1;
      LevelView<T> vc = view<T>(h, lc);
      const size_t nc3 = 3 * (size_t)vc.N * vc.N;
      if (f32) {
        T* bb2 = h->p<T>(lc == 0 ? h->b0f : h->L[lc].b);
        T* ww = h->p<T>(lc == 0 ? h->w0f : h->L[lc].w);
        k_convert<double, T><<<nblk(nc3), 256, 0, s>>>(a, bb2, nc3);
        launch_coarse_apply<T>(s, h->p<double>(h->cainv), h->nr, bb2, ww);
        k_convert<T, double><<<nblk(nc3), 256, 0, s>>>(ww, out, nc3);
      } else {
        launch_coarse_apply<T>(s, h->p<double>(h->cainv), h->nr, (const T*)a, (T*)out);
      }
      break;
    }
    default: return IBMG_EINVAL;
  }
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

int single(ibmg_handle* h, int which, int level, const double* a, const double* b, double* out, int sweeps) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  return h->prec == IBMG_FP32 ? single_op<float>(h, which, level, a, b, out, sweeps)
                              : single_op<double>(h, which, level, a, b, out, sweeps);
}

}  // namespace

extern "C" {

int ibmg_apply(ibmg_handle* h, int level, const double* w, double* y) {
  if (!w || !y) return IBMG_EINVAL;
  return single(h, 0, level, w, nullptr, y, 0);
}
int ibmg_residual(ibmg_handle* h, int level, const double* b, const double* w, double* r) {
  if (!w || !b || !r) return IBMG_EINVAL;
  return single(h, 1, level, w, b, r, 0);
}
int ibmg_smooth(ibmg_handle* h, int level, const double* b, double* w, int sweeps) {
  if (!w || !b || sweeps < 0) return IBMG_EINVAL;
  return single(h, 2, level, nullptr, b, w, sweeps);
}
int ibmg_restrict(ibmg_handle* h, int level, const double* fine, double* coarse) {
  if (!fine || !coarse) return IBMG_EINVAL;
  return single(h, 3, level, fine, nullptr, coarse, 0);
}
int ibmg_prolong_add(ibmg_handle* h, int level, const double* coarse, double* fine) {
  if (!fine || !coarse) return IBMG_EINVAL;
  return single(h, 4, level, coarse, nullptr, fine, 0);
}
int ibmg_coarse_solve(ibmg_handle* h, const double* b, double* w) {
  if (!b || !w) return IBMG_EINVAL;
  return single(h, 5, 0, b, nullptr, w, 0);
}

int ibmg_vcycle(ibmg_handle* h, const double* r, double* z) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (!r || !z) return IBMG_EINVAL;
  precond(h, r, z);
  if (h->launch_error) return IBMG_EHIP;
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

int ibmg_box_matrix(ibmg_handle* h, int level, int bx, int by, double* out) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!h->setup_ok) return IBMG_ESTATE;
  if (!out || level < 0 || level >= h->levels - 1) return IBMG_EINVAL;
  const LevelBufs& B = h->L[level];
  if (bx < 0 || by < 0 || bx >= B.nb || by >= B.nb) return IBMG_EINVAL;
  LevelView<double> v = view<double>(h, level);
  launch_box_matrix(h->stream, v, bx, by, out);
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

int ibmg_fiber_force(ibmg_handle* h, const double* X, double* G) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (h->M == 0) return IBMG_OK;
  if (!X || !G) return IBMG_EINVAL;
  launch_fiber_force(h->stream, h->M, h->p<int>(h->prev_d), h->p<int>(h->next_d), h->K, X, G);
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

}  // extern "C"

namespace {
// Finest-level point data (weights and box lists) for arbitrary X.
int fine_points(ibmg_handle* h, const double* X) {
  hipStream_t s = h->stream;
  h->setup_ok = false;
  launch_weights0(s, h->M, h->N, h->kind, X, h->p<int>(h->org), h->p<double>(h->wts));
  launch_box_lists(s, points(h), h->p<int>(h->cnt), h->p<int>(h->start), h->p<int>(h->cursor), h->p<int>(h->list),
                   h->max_list, h->p<int>(h->ltotal), h->p<int>(h->loc), h->p<int>(h->bsum));
  IBMG_HIP(hipGetLastError());
  return IBMG_OK;
}
}  // namespace

extern "C" {

int ibmg_spread(ibmg_handle* h, const double* X, const double* G, double* fu, double* fv) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (!fu || !fv || (h->M > 0 && (!X || !G))) return IBMG_EINVAL;
  const size_t NN = (size_t)h->N * h->N;
  double* b = h->p<double>(h->bvec);
  if (h->M > 0) {
    int rc = fine_points(h, X);
    if (rc) return rc;
  }
  launch_rhs(h->stream, points(h), 0.0, (double)h->N * h->N, nullptr, nullptr, nullptr, nullptr, h->M > 0 ? G : nullptr,
             b);
  IBMG_HIP(hipMemcpyAsync(fu, b, NN * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  IBMG_HIP(hipMemcpyAsync(fv, b + NN, NN * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

int ibmg_interp(ibmg_handle* h, const double* X, const double* u, const double* v, double* U) {
  if (!ready(h)) return IBMG_ENOMEM;
  if (h->M == 0) return IBMG_OK;
  if (!X || !u || !v || !U) return IBMG_EINVAL;
  int rc = fine_points(h, X);
  if (rc) return rc;
  launch_interp(h->stream, points(h), u, v, U, nullptr, 0.0);
  IBMG_HIP(hipGetLastError());
  return sync(h);
}

}  // extern "C"
