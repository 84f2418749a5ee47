// Internal host-side state shared by the single-problem ABI (api.hip) and
// the batched ABI (batch.hip): the handle, its workspace layout and the
// level views handed to the kernels.
#pragma once
#include <mutex>
#include <vector>

#include "../../include/ibmg.h"
#include "common.h"

namespace ibmg {

constexpr int kPW = 16;          // panel width of the coarse Gauss-Jordan (dense.hip)
constexpr int kDotBlocks = 256;  // workgroups of the deterministic dot products
constexpr int kMaxTimed = 8192;  // timed phase launches per solve
constexpr int kFallbackWindow = 20;  // FP32 V-cycle stall test: < 10% progress over this many iterations
constexpr int kMaxBasis = 1000;     // largest Krylov basis (restart length)
constexpr int kMaxIters = 1000000;  // largest iteration cap with restarts
constexpr int kSmallLevel = 32;  // default (and largest) level size run in one workgroup per V-cycle leg

struct Buf {
  size_t off = 0, bytes = 0;
};

struct LevelBufs {
  int N = 0, nb = 0, maxact = 0, reach = 0;
  Buf w, b, r;               // V-cycle vectors in the V-cycle precision
  Buf act, rows, nact;       // active elastic rows of this level
  Buf win, winf;             // FP64 windows and their FP32 copy
  Buf yib;                   // elastic rows evaluated before a colour phase (V-cycle precision)
  Buf crow, ncrow;           // one-launch four-colour levels: active rows in the boxes of each colour
  Buf ib_index, ib_boxes, boxflag, info;
  Buf ainv_plain, ainv_plain_f, ainv_ib;
  int max_ib = 0;
  int rowhint = 0;           // launch-size hint of the elastic-row passes (see LevelView)
};

}  // namespace ibmg

using ibmg::Buf;
using ibmg::LevelBufs;

struct ibmg_handle {
  // problem and options
  int N = 0, M = 0, nfib = 0, kind = 0, levels = 0, n = 4, nu1 = 2, nu2 = 2, maxit = 100, prec = 0, guess = 0;
  int ncol = 2;
  int ncol_l[IBMG_MAX_LEVELS] = {};   // colour classes of each level's sweeps
  int scheme = 0; // IBMG_IMPLICIT or IBMG_EXPLICIT
  int solver = 0; // IBMG_SOLVER_FGMRES or IBMG_SOLVER_MG
  double omega = 1.0;  // box correction weight
  int orth = 0;        // IBMG_ORTH_CGS2 or IBMG_ORTH_DCGS2
  int mb = 100;   // Krylov basis size: the FGMRES(m) restart length (maxit caps the iterations of all cycles)
  int tail_max = ibmg::kSmallLevel;   // largest level size run by the LDS-resident tail
  double rho = 1, mu = 1, K = 0, rtol = 1e-8;
  std::vector<int> prev, next;
  hipStream_t stream = nullptr;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  LevelBufs L[IBMG_MAX_LEVELS];
  Buf X0, G, prev_d, next_d, U;
  Buf org, wts, cnt, start, cursor, list, ltotal;   // finest-level point data and bins
  Buf flag, loc, bsum, meta;                        // scan scratch and setup flags
  int max_list = 0;
  Buf V, Z, H, g, cs, sn, y, flags, partial, scal, hc;
  Buf bvec, xvec, rvec, w0f, b0f;
  Buf xbest;   // iterate with the smallest true residual of the solve so far
  Buf aug, cm, cpiv, crowpos, cused, cY, cainv;
  int nr = 0, ndof = 0;
  // state
  bool setup_ok = false, has_ib = false, launch_error = false;
  bool walls = false;   // IBMG_CAVITY: walls on all four sides, the top one moving (Sec. 4)
  // boxes that take their own inverse: those with elastic rows, and with
  // walls the boxes touching a wall
  bool own_boxes() const { return has_ib || walls; }
  bool fb64 = false;   // this solve continues with the FP64 V-cycle (FP32 stalled)
  bool yib64 = false;  // FP32 handle: the FP64 V-cycle left FP64 values in the elastic-row buffers
  // the V-cycle as a captured graph (fixed buffers b0g -> w0g), rebuilt when dt changes
  hipStream_t cap = nullptr;
  double* flags_h = nullptr;   // pinned host memory the Givens kernel writes its flags into
  double* flags_d = nullptr;   // the same memory as the device addresses it
  hipEvent_t flag_ev[2] = {nullptr, nullptr};   // marks each slot's flags as written
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_dt = -1.0;
  Buf b0g, w0g;
  double dt = 0;
  int n_ib[IBMG_MAX_LEVELS][5] = {};
  // setup counts read back between setup_launch and setup_finish
  std::vector<int> rb_info, rb_nact, rb_mt, rb_lt;
  // timing of the box-relaxation phase kernel
  bool timing = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  std::vector<double> ev_bytes;
  double t_total_ms = 0, t_bytes = 0;
  int64_t t_launches = 0;

  template <typename T> T* p(const Buf& b) const { return reinterpret_cast<T*>(ws + b.off); }
  size_t n0() const { return 3 * (size_t)N * N; }
};

namespace ibmg {

template <typename T>
inline LevelView<T> view(const ibmg_handle* h, int l) {
  const LevelBufs& B = h->L[l];
  LevelView<T> v{};
  v.N = B.N;
  v.nb = B.nb;
  v.n = h->n;
  v.ndof = h->ndof;
  v.ncol = h->ncol_l[l];
  const double hl = 1.0 / B.N;
  v.c = (T)(h->rho / h->dt);
  v.muh2 = (T)(h->mu / (hl * hl));
  v.invh = (T)(1.0 / hl);
  v.omega = (T)h->omega;
  v.walls = h->walls ? 1 : 0;
  v.reach = B.reach;
  v.maxact = B.maxact;
  v.rowhint = B.rowhint > 0 ? B.rowhint : B.maxact;
  if (h->has_ib) {
    v.act = h->p<int>(B.act);
    v.rows = h->p<int>(B.rows);
    v.nact = h->p<int>(B.nact);
    v.yib = h->p<T>(B.yib);
    if (B.crow.bytes) {
      v.crow = h->p<int>(B.crow);
      v.ncrow = h->p<int>(B.ncrow);
    }
    v.win = sizeof(T) == sizeof(float) ? reinterpret_cast<const T*>(h->p<float>(B.winf))
                                       : reinterpret_cast<const T*>(h->p<double>(B.win));
  }
  if (l < h->levels - 1) {
    v.ib_index = h->p<int>(B.ib_index);
    v.ainv_plain = sizeof(T) == sizeof(float) ? reinterpret_cast<const T*>(h->p<float>(B.ainv_plain_f))
                                              : reinterpret_cast<const T*>(h->p<double>(B.ainv_plain));
    v.ainv_ib = h->p<double>(B.ainv_ib);
  }
  return v;
}

inline PointView points(const ibmg_handle* h) {
  PointView P{};
  P.M = h->M;
  P.N = h->N;
  P.n = h->n;
  P.nb = h->L[0].nb;
  P.prev = h->p<int>(h->prev_d);
  P.next = h->p<int>(h->next_d);
  P.org = h->p<int>(h->org);
  P.wts = h->p<double>(h->wts);
  P.box_start = h->p<int>(h->start);
  P.box_list = h->p<int>(h->list);
  return P;
}

// First level handled by the LDS-resident tail of the V-cycle: every level
// from there down has at most tail_max cells per side.
inline int tail_start(const ibmg_handle* h) {
  int ls = h->levels - 1;
  if (h->n > 4) return ls;   // 8 x 8 boxes: the plain inverse does not fit the tail's LDS
  while (ls > 0 && h->L[ls - 1].N <= h->tail_max) --ls;
  return ls;
}

// Dynamic LDS of the tail: three vectors (nine arrays) per level from ls on,
// and one plain-box inverse.
inline size_t tail_lds(const ibmg_handle* h, size_t elem) {
  const int ls = tail_start(h);
  // a tail of the coarsest level alone (the batched V-cycle runs it in the
  // tail kernel) smooths nothing and stages no box inverse
  size_t lds = ls < h->levels - 1 ? (size_t)h->ndof * h->ndof * elem : 0;
  for (int l = ls; l < h->levels; ++l) lds += 9 * (size_t)h->L[l].N * h->L[l].N * elem;
  return lds;
}

// Graph capture and instantiation are serialised over the process: handles
// driven from several host threads (one stream each) then never capture or
// instantiate at the same time.  The HIP runtime allows concurrent
// thread-local captures, but a kernel-tracing profiler that intercepts the
// capture and instantiate calls faulted on the host when eight threads did so
// together; the lock costs nothing outside that moment (captures happen once
// per time-step size or when the active set outgrows a captured launch).
inline std::mutex& capture_mutex() {
  static std::mutex m;
  return m;
}

void layout(ibmg_handle* h);
int bind(ibmg_handle* h, void* dev, size_t bytes, bool own_capture_stream);
int setup_launch(ibmg_handle* h, double dt, const double* X);
int setup_finish(ibmg_handle* h);
int step_begin(ibmg_handle* h, double dt, const double* u, const double* v, const double* p, const double* gu,
               const double* gv);
int step_end(ibmg_handle* h, double dt, double* u, double* v, double* p, double* X);
// z = MGV(0, r) with the FP64 V-cycle, launched eagerly on the handle's stream.
void vcycle_fp64(ibmg_handle* h, const double* r, double* z);
// Before an FP32 V-cycle or smoothing pass on an FP32 handle: clears the
// elastic-row buffers if an FP64 fallback V-cycle has used them since setup.
void yib_for_fp32(ibmg_handle* h);

}  // namespace ibmg
