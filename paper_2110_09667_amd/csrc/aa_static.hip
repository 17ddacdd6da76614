// aa_static.hip -- the least-squares solve R gamma = Q^T f (Alg. 2, last
// line) for callers that cannot allocate device memory and hold no context:
// its reduction partials live in a file-scope device array of fixed size
// instead of a workspace, and nothing here allocates.
#include <mutex>

#include "aa_internal.h"

using namespace aa;

namespace {

// Streaming workgroups of the dot-product pass (as the context's default) and
// the partials they publish: k values per workgroup, k <= 64.
constexpr int kStaticGrid = 512;
constexpr int kStaticMaxK = 64;
constexpr size_t kStaticPartials = (size_t)kStaticMaxK * kStaticGrid;
// after the partials: c (64), scalars (S_COUNT) and the status word
constexpr size_t kStaticDoubles = kStaticPartials + kStaticMaxK + S_COUNT + 8;

}  // namespace

// One copy per GPU, held until the process ends (about 257 KiB).  Host code
// never uses this name as an address: it asks for each device's address once.
static __device__ __align__(256) double scratch[kStaticDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device with that device current); nullptr on failure.
double* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = (double*)p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" aa_status aa_qr_solve_noalloc(const double* d_Q, int64_t ldq, int64_t n, int k,
                                         const double* d_R, int ldr, const double* d_f,
                                         double* d_gamma, void* stream) {
  if (!d_Q || !d_R || !d_f || !d_gamma || n < 1 || ldq < n || k < 1 || k > kStaticMaxK ||
      ldr < k)
    return AA_EINVAL;
  double* base = scratch_on_current_device();
  if (!base) return AA_EHIP;
  Small sm{};
  sm.R = const_cast<double*>(d_R);  // read only by the back substitution
  sm.T = nullptr;
  sm.coef0 = nullptr;
  sm.coef1 = base + kStaticPartials;  // c = Q^T f (written by the tail)
  sm.gamma = d_gamma;
  sm.givens = nullptr;
  sm.scal = base + kStaticPartials + kStaticMaxK;
  sm.status = (int*)(base + kStaticPartials + kStaticMaxK + S_COUNT);
  sm.partials = base;
  sm.cap = ldr;
  int64_t g = (n + kTile - 1) / kTile;
  const int grid = (int)(g > kStaticGrid ? kStaticGrid : (g < 1 ? 1 : g));
  DotsArgs d{d_Q, ldq, n, d_f, k, nullptr, 0, 0};
  Tail t{};
  t.op = TAIL_RHS;
  t.k = k;
  // every partial the pass publishes (k per workgroup) is written before the
  // finalize reads it, so nothing of an earlier call needs clearing
  return launch_dots(d, sm, t, grid, (hipStream_t)stream) == hipSuccess ? AA_OK : AA_EHIP;
}
