// ibmg_spread_noalloc: the force spreading of ibmg_spread (Sec. 2.2,
// f = S_0 G through the 4-point regularised delta, deterministic gather over
// points binned by box) for callers that cannot allocate device memory.  Its
// kernels are the ones ibmg_spread launches; their scratch (patch origins and
// weights, box bins, scan partials, the stacked right-hand side) lives in one
// file-scope device array instead of a handle's workspace.
//
// The array is per GPU: each device holds its own copy at its own address,
// taken once per device with hipGetSymbolAddress (the array's name in host
// code is a host-side stand-in, never passed to a kernel or a copy).  Every
// call on a device shares that device's copy and leaves its contents behind,
// so calls that overlap on one GPU (two streams, two threads) race; the bins
// are cleared by the kernels themselves at the start of every call.
#include <mutex>

#include "../../include/ibmg.h"
#include "common.h"
#include "kernels.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // 16 MiB per GPU
constexpr int kNoAllocMaxN = 512, kNoAllocMinN = 16, kNoAllocMaxM = 8192;
constexpr int kNoAllocBox = 4;    // bin size in cells (the default box edge)
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
char* g_scratch[kMaxDevices] = {};

size_t carve(size_t& cur, size_t bytes) {
  cur = (cur + 255) & ~(size_t)255;
  const size_t off = cur;
  cur += bytes;
  return off;
}

// Offsets of the scratch regions for an N x N grid and M points; returns the
// bytes needed.
struct Layout {
  size_t org, wts, cnt, start, cursor, list, total, loc, bsum, b, need;
  int max_list;
};

Layout layout_for(int N, int M) {
  Layout L{};
  size_t cur = 0;
  const int nb = N / kNoAllocBox, nbox = nb * nb;
  const int a = (4 + kNoAllocBox - 1) / kNoAllocBox + 2;   // boxes a point's 4 x 4 patches can touch, per side
  const size_t Mx = M > 0 ? (size_t)M : 1;
  L.max_list = (int)(Mx * a * a);
  L.org = carve(cur, 4 * Mx * sizeof(int));
  L.wts = carve(cur, 2 * Mx * IBMG_PATCH * sizeof(double));
  L.cnt = carve(cur, (nbox + 1) * sizeof(int));
  L.start = carve(cur, (nbox + 1) * sizeof(int));
  L.cursor = carve(cur, nbox * sizeof(int));
  L.list = carve(cur, (size_t)L.max_list * sizeof(int));
  L.total = carve(cur, 4 * sizeof(int));
  L.loc = carve(cur, (nbox + 1) * sizeof(int));
  L.bsum = carve(cur, ((nbox + 1) / 1024 + 2) * sizeof(int));
  L.b = carve(cur, 3 * (size_t)N * N * sizeof(double));
  L.need = cur;
  return L;
}

// The device address of this device's scratch array (taken on first use).
int scratch_base(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return IBMG_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return IBMG_EHIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IBMG_EHIP;
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return IBMG_OK;
}

}  // namespace

extern "C" int ibmg_spread_noalloc(int32_t N, int32_t delta, int32_t M, const double* X, const double* G,
                                   double* f_u, double* f_v, void* stream) {
  using namespace ibmg;
  if (N < kNoAllocMinN || N > kNoAllocMaxN || (N & (N - 1)) != 0) return IBMG_EINVAL;
  if (M < 0 || M > kNoAllocMaxM) return IBMG_EINVAL;
  if (delta != IBMG_DELTA_IB4 && delta != IBMG_DELTA_COS4) return IBMG_EINVAL;
  if (!f_u || !f_v || (M > 0 && (!X || !G))) return IBMG_EINVAL;
  const Layout Lo = layout_for(N, M);
  if (Lo.need > kScratchBytes) return IBMG_EINVAL;
  char* base = nullptr;
  const int rc = scratch_base(&base);
  if (rc != IBMG_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* org = reinterpret_cast<int*>(base + Lo.org);
  double* wts = reinterpret_cast<double*>(base + Lo.wts);
  PointView P{};
  P.M = M;
  P.N = N;
  P.n = kNoAllocBox;
  P.nb = N / kNoAllocBox;
  P.org = org;
  P.wts = wts;
  P.box_start = reinterpret_cast<int*>(base + Lo.start);
  P.box_list = reinterpret_cast<int*>(base + Lo.list);
  double* b = reinterpret_cast<double*>(base + Lo.b);
  launch_weights0(s, M, N, delta, X, org, wts);
  launch_box_lists(s, P, reinterpret_cast<int*>(base + Lo.cnt), reinterpret_cast<int*>(base + Lo.start),
                   reinterpret_cast<int*>(base + Lo.cursor), reinterpret_cast<int*>(base + Lo.list), Lo.max_list,
                   reinterpret_cast<int*>(base + Lo.total), reinterpret_cast<int*>(base + Lo.loc),
                   reinterpret_cast<int*>(base + Lo.bsum));
  launch_rhs(s, P, 0.0, (double)N * N, nullptr, nullptr, nullptr, nullptr, M > 0 ? G : nullptr, b);
  const size_t NN = (size_t)N * N;
  if (hipMemcpyAsync(f_u, b, NN * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return IBMG_EHIP;
  if (hipMemcpyAsync(f_v, b + NN, NN * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return IBMG_EHIP;
  if (hipGetLastError() != hipSuccess) return IBMG_EHIP;
  return IBMG_OK;
}
