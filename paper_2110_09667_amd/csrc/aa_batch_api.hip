// aa_batch_api.hip -- host side of the batched C ABI (aa_batch_* in aa.h).
//
// The workspace holds the instance descriptors, their device-updated states,
// the schedule (instance order and work counter) and, per instance, G(x),
// f_{i-1}, G(x_{i-1}), Delta f, Q, the Delta g history and the small dense
// block.  aa_batch_run enqueues one persistent launch per iteration (after a
// one-thread reset of the work counter); with a non-NULL stream the sequence
// for a given iteration count is captured once as a HIP graph and replayed.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "aa_internal.h"

using namespace aa;

struct aa_batch {
  int count = 0, variant = 0;
  unsigned flags = 0;
  double tol = 0.0;
  int64_t max_iter = 0;
  hipStream_t stream = nullptr;
  BInst* d_inst = nullptr;
  BState* d_state = nullptr;
  int* d_order = nullptr;
  unsigned* d_counter = nullptr;
  std::vector<int64_t> n;
  std::vector<int> m;
  std::vector<int> dim;
  int kbucket = 8;
  int mmax = 1;         // largest window of the batch
  bool gram = false;
  int grid = 0;        // persistent workgroups (0: 2 per compute unit)
  int order_mode = 0;  // 0: largest n*m first, 1: as given
  bool use_graph = true;
  hipGraphExec_t exec = nullptr;
  int exec_iters = 0;
  bool learned = false;
  float* d_feat = nullptr;  // [count x AA_MLP_FEATURES]
  float* d_out = nullptr;   // [count x AA_MLP_OUTPUTS]
  float* d_dout = nullptr;  // [count x AA_MLP_OUTPUTS]
  int pairs = 4;            // row pairs per lane per tile of the persistent kernel
  // split path: once few instances are active, the large ones leave the
  // persistent kernel and run on the grid-wide passes (many workgroups each)
  int64_t split_min_n = 65536;  // 0: never
  int split_active_max = 0;     // split when at most this many are active (0: CUs / 4)
  int* d_skip = nullptr;        // [count] 1: left out of the persistent kernel
  StopState* d_stops = nullptr; // [count] stop state of a split instance
  double* d_partials = nullptr; // shared by the split instances' passes
  std::vector<BInst> hinst;     // host copies of the descriptors
  std::vector<int> split;       // instances on the split path
  std::vector<aa_ctx*> views;   // their contexts
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ld_of(int64_t n) { return (n + 63) / 64 * 64; }

bool valid_instance(const aa_batch_instance& I) {
  if (I.m < 1 || I.m > 64 || I.dim < 1 || I.dim > 3 || I.s < 1) return false;
  int64_t n = I.s;
  if (I.dim >= 2) n *= I.s;
  if (I.dim >= 3) n *= I.s;
  if (n != I.n || !(I.h > 0.0) || !I.d_f || !I.d_x) return false;
  if (((uintptr_t)I.d_f % 16) != 0 || ((uintptr_t)I.d_x % 16) != 0) return false;
  return true;
}

size_t instance_bytes(int64_t n, int m, bool learned) {
  const size_t vec = align_up((size_t)ld_of(n) * sizeof(double));
  size_t b = (learned ? 6 : 4) * vec + 2 * (size_t)m * vec;  // g, f_prev, g_prev, W, (xc, gc), Q, ring
  b += 2 * align_up(sizeof(double) * m * m);  // R, T
  b += 3 * align_up(sizeof(double) * m);      // coef0, coef1, gamma
  b += align_up(sizeof(double) * 2 * m);      // Givens
  b += align_up(sizeof(double) * S_COUNT);    // scalars
  b += align_up(sizeof(int));                 // status
  return b;
}

// Reduction partials of one grid-wide pass (the split path's passes run one
// after another and share them): 199 values x 8192 workgroups, as a
// single-instance context holds.
constexpr size_t kSplitPartials = (size_t)(3 * AA_MAX_COLS + 4) * 8192;

size_t header_bytes(int count, bool learned) {
  size_t b = align_up(sizeof(BInst) * count) + align_up(sizeof(BState) * count) +
             align_up(sizeof(int) * count) + align_up(sizeof(unsigned));
  b += align_up(sizeof(int) * count) + align_up(sizeof(StopState) * count) +
       align_up(sizeof(double) * kSplitPartials);
  if (learned)
    b += align_up(sizeof(float) * count * kFeat) + 2 * align_up(sizeof(float) * count * kOuts);
  return b;
}

int bucket(int m) { return m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64; }

void drop_graph(aa_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->exec_iters = 0;
}

hipError_t enqueue_mode(aa_batch* b, int mode, float dscale) {
  BatchArgs a{};
  a.inst = b->d_inst;
  a.state = b->d_state;
  a.order = b->d_order;
  a.count = b->count;
  a.counter = b->d_counter;
  a.variant = b->variant;
  a.flags = b->flags;
  a.tol = b->tol;
  a.max_iter = b->max_iter;
  a.ov_iter = -1;
  a.mode = mode;
  a.skip = mode == BM_PLAIN && !b->split.empty() ? b->d_skip : nullptr;
  a.feat = b->d_feat;
  a.out = b->d_out;
  a.dout = b->d_dout;
  a.dscale = dscale;
  int grid = b->grid;
  if (grid <= 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    grid = 2 * cus;
  }
  if (grid > b->count) grid = b->count;
  hipError_t e = launch_batch_reset(b->d_counter, b->stream);
  if (e != hipSuccess) return e;
  return launch_batch(a, grid, b->kbucket, b->gram,
                      batch_stage_cols(b->mmax, b->variant, b->flags), b->stream, b->pairs);
}

// One iteration of every split instance on the grid-wide passes: G by the
// stencil kernel, aa_step on the instance's view, then its batched state.
hipError_t enqueue_split(aa_batch* b) {
  for (size_t t = 0; t < b->split.size(); ++t) {
    const int j = b->split[t];
    const BInst& I = b->hinst[j];
    hipError_t e = launch_stencil(I.dim, I.s, I.h, I.omega, I.c, I.f, I.x, I.g, b->stream);
    if (e != hipSuccess) return e;
    if (aa_step(b->views[t], I.x, I.g, I.x) != AA_OK) return hipErrorUnknown;
    int64_t it = 0;
    int k = 0, mi = 0;
    view_counters(b->views[t], &it, &k, &mi);
    e = launch_split_state(b->d_state + j, b->d_stops + j, I.sm, k, mi, b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Return every split instance to the persistent kernel (its memory layout is
// the same on both paths).
hipError_t merge_split(aa_batch* b) {
  if (b->split.empty()) return hipSuccess;
  for (aa_ctx* v : b->views) view_destroy(v);
  b->views.clear();
  b->split.clear();
  return launch_set_int(b->d_skip, b->count, 0, b->stream);
}

// Split policy, evaluated when a run starts: once at most split_active_max
// instances are active (the persistent kernel no longer fills the chip), the
// active instances with n >= split_min_n leave it for the grid-wide passes;
// split instances that have stopped are dropped from the list.
aa_status update_split(aa_batch* b) {
  if (b->split_min_n <= 0) return AA_OK;
  std::vector<BState> hs(b->count);
  if (hipMemcpyAsync(hs.data(), b->d_state, sizeof(BState) * b->count, hipMemcpyDeviceToHost,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return AA_EHIP;
  for (size_t t = 0; t < b->split.size();) {
    if (!hs[b->split[t]].active) {
      view_destroy(b->views[t]);
      b->views.erase(b->views.begin() + t);
      b->split.erase(b->split.begin() + t);
    } else {
      ++t;
    }
  }
  int active = 0;
  for (const BState& st : hs) active += st.active ? 1 : 0;
  int amax = b->split_active_max;
  if (amax <= 0) {
    // measured crossover of the 2D table's largest instances (n ~ 1.5e5 to
    // 2.6e5): one workgroup streams ~19 GB/s, one instance on the grid-wide
    // passes ~1.4 TB/s (launch-bound at that n); below ~80 active instances
    // the split path wins
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    amax = cus / 4 > 1 ? cus / 4 : 1;
  }
  if (active == 0 || active > amax) return AA_OK;
  std::vector<int> add;
  for (int j = 0; j < b->count; ++j)
    if (hs[j].active && !hs[j].pending && hs[j].iter >= 1 && b->n[j] >= b->split_min_n &&
        std::find(b->split.begin(), b->split.end(), j) == b->split.end())
      add.push_back(j);
  for (int j : add) {
    const BState& st = hs[j];
    StopState s0{};
    s0.done = 0;
    s0.cur = st.iter;
    if (hipMemcpyAsync(b->d_stops + j, &s0, sizeof(s0), hipMemcpyHostToDevice, b->stream) !=
        hipSuccess)
      return AA_EHIP;
    const int one = 1;
    if (hipMemcpyAsync(b->d_skip + j, &one, sizeof(int), hipMemcpyHostToDevice, b->stream) !=
        hipSuccess)
      return AA_EHIP;
    aa_ctx* v = view_create(b->hinst[j], b->variant, b->flags, b->d_partials, b->d_stops + j,
                            st.iter, st.k, st.m_i, b->tol, b->max_iter, b->stream);
    if (!v) return AA_EINVAL;
    b->split.push_back(j);
    b->views.push_back(v);
  }
  if (!add.empty()) drop_graph(b);
  return hipStreamSynchronize(b->stream) == hipSuccess ? AA_OK : AA_EHIP;
}

hipError_t enqueue(aa_batch* b, int iters) {
  for (int i = 0; i < iters; ++i) {
    hipError_t e = enqueue_mode(b, BM_PLAIN, 0.f);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

aa_status aa_batch_workspace_size(int count, const aa_batch_instance* inst, int variant,
                                  unsigned flags, size_t* bytes) {
  if (count < 1 || !inst || !bytes || variant < AA_MGS || variant > AA_ICWY) return AA_EINVAL;
  if (flags & AA_ICWY_T_TRANSFORM) return AA_EINVAL;  // one-workgroup step: Gram refresh only
  const bool learned = (flags & AA_BATCH_LEARNED) != 0;
  size_t tot = header_bytes(count, learned);
  for (int j = 0; j < count; ++j) {
    if (!valid_instance(inst[j])) return AA_EINVAL;
    if (learned && inst[j].m > kWin) return AA_EINVAL;  // features cover a 20-column window
    tot += instance_bytes(inst[j].n, inst[j].m, learned);
  }
  *bytes = tot;
  return AA_OK;
}

aa_status aa_batch_init(aa_batch** out, int count, const aa_batch_instance* inst, int variant,
                        unsigned flags, double tol, int64_t max_iter, void* d_ws,
                        size_t bytes, void* stream) {
  if (!out) return AA_EINVAL;
  *out = nullptr;
  size_t need = 0;
  aa_status s = aa_batch_workspace_size(count, inst, variant, flags, &need);
  if (s != AA_OK) return s;
  if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || !(tol >= 0.0) || max_iter < 1)
    return AA_EINVAL;
  if (bytes < need) return AA_ENOSPACE;
  aa_batch* b = new (std::nothrow) aa_batch();
  if (!b) return AA_EINVAL;
  b->count = count;
  b->variant = variant;
  b->flags = flags;
  b->tol = tol;
  b->max_iter = max_iter;
  b->stream = (hipStream_t)stream;
  char* base = (char*)d_ws;
  size_t o = 0;
  b->d_inst = (BInst*)(base + o); o = align_up(o + sizeof(BInst) * count);
  b->d_state = (BState*)(base + o); o = align_up(o + sizeof(BState) * count);
  b->d_order = (int*)(base + o); o = align_up(o + sizeof(int) * count);
  b->d_counter = (unsigned*)(base + o); o = align_up(o + sizeof(unsigned));
  b->d_skip = (int*)(base + o); o = align_up(o + sizeof(int) * count);
  b->d_stops = (StopState*)(base + o); o = align_up(o + sizeof(StopState) * count);
  b->d_partials = (double*)(base + o); o = align_up(o + sizeof(double) * kSplitPartials);
  b->learned = (flags & AA_BATCH_LEARNED) != 0;
  if (b->learned) {
    b->d_feat = (float*)(base + o); o = align_up(o + sizeof(float) * count * kFeat);
    b->d_out = (float*)(base + o); o = align_up(o + sizeof(float) * count * kOuts);
    b->d_dout = (float*)(base + o); o = align_up(o + sizeof(float) * count * kOuts);
  }
  std::vector<BInst> hi(count);
  std::vector<BState> hs(count);
  int mmax = 1;
  for (int j = 0; j < count; ++j) {
    const aa_batch_instance& A = inst[j];
    BInst& I = hi[j];
    const int64_t ld = ld_of(A.n);
    const size_t vec = align_up((size_t)ld * sizeof(double));
    const int m = A.m;
    I.n = A.n; I.ld = ld; I.m = m; I.dim = A.dim; I.s = A.s;
    I.h = A.h; I.omega = A.omega; I.c = A.c;
    I.f = A.d_f; I.x = A.d_x;
    I.g = (double*)(base + o); o += vec;
    I.f_prev = (double*)(base + o); o += vec;
    I.g_prev = (double*)(base + o); o += vec;
    I.W = (double*)(base + o); o += vec;
    if (b->learned) {
      I.xc = (double*)(base + o); o += vec;
      I.gc = (double*)(base + o); o += vec;
    }
    I.Q = (double*)(base + o); o += vec * m;
    I.ring = (double*)(base + o); o += vec * m;
    Small& sm = I.sm;
    sm.R = (double*)(base + o); o = align_up(o + sizeof(double) * m * m);
    sm.T = (double*)(base + o); o = align_up(o + sizeof(double) * m * m);
    sm.coef0 = (double*)(base + o); o = align_up(o + sizeof(double) * m);
    sm.coef1 = (double*)(base + o); o = align_up(o + sizeof(double) * m);
    sm.gamma = (double*)(base + o); o = align_up(o + sizeof(double) * m);
    sm.givens = (double*)(base + o); o = align_up(o + sizeof(double) * 2 * m);
    sm.scal = (double*)(base + o); o = align_up(o + sizeof(double) * S_COUNT);
    sm.status = (int*)(base + o); o = align_up(o + sizeof(int));
    sm.partials = nullptr;
    sm.cap = m;
    sm.stop = nullptr;  // batched instances stop by their own per-instance test
    BState& st = hs[j];
    st.iter = 0; st.conv_iter = -1; st.k = 0; st.m_i = 0; st.active = 1; st.status = 0;
    st.res_norm = st.res0_norm = 0.0;
    st.g_evals = st.accepted = 0;
    st.loss = 0.0;
    st.pending = st.g_valid = 0;
    b->n.push_back(A.n);
    b->m.push_back(m);
    b->dim.push_back(A.dim);
    mmax = std::max(mmax, m);
  }
  b->kbucket = bucket(mmax);
  b->mmax = mmax;
  b->gram = batch_needs_gram(variant, flags);
  hipError_t e = hipMemcpyAsync(b->d_inst, hi.data(), sizeof(BInst) * count,
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_state, hs.data(), sizeof(BState) * count, hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = launch_batch_init(b->d_inst, count, b->stream);
  if (e == hipSuccess) e = launch_set_int(b->d_skip, count, 0, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  b->hinst = hi;
  if (e != hipSuccess) {
    delete b;
    return AA_EHIP;
  }
  if (aa_batch_set_schedule(b, 0, 0, 1) != AA_OK) {
    delete b;
    return AA_EHIP;
  }
  *out = b;
  return AA_OK;
}

aa_status aa_batch_set_schedule(aa_batch* b, int grid, int order, int use_graph) {
  if (!b || grid < 0 || grid > 65536 || order < 0 || order > 1) return AA_EINVAL;
  std::vector<int> ord(b->count);
  std::iota(ord.begin(), ord.end(), 0);
  if (order == 0)
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
      return b->n[a] * b->m[a] > b->n[c] * b->m[c];
    });
  if (hipMemcpyAsync(b->d_order, ord.data(), sizeof(int) * b->count, hipMemcpyHostToDevice,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return AA_EHIP;
  b->grid = grid;
  b->order_mode = order;
  b->use_graph = use_graph != 0;
  drop_graph(b);
  return AA_OK;
}

aa_status aa_batch_set_split(aa_batch* b, int64_t min_n, int active_max) {
  if (!b || min_n < 0 || active_max < 0) return AA_EINVAL;
  b->split_min_n = min_n;
  b->split_active_max = active_max;
  if (min_n == 0 && merge_split(b) != hipSuccess) return AA_EHIP;
  return AA_OK;
}

aa_status aa_batch_split_count(const aa_batch* b, int* count) {
  if (!b || !count) return AA_EINVAL;
  *count = (int)b->split.size();
  return AA_OK;
}

aa_status aa_batch_set_tiles(aa_batch* b, int pairs) {
  if (!b || (pairs != 2 && pairs != 4)) return AA_EINVAL;
  b->pairs = pairs;
  drop_graph(b);
  return AA_OK;
}

aa_status aa_batch_autotune(aa_batch* b, int iters, const char* cache_path,
                            aa_batch_schedule* best) {
  if (!b || iters < 1) return AA_EINVAL;
  // candidates are timed on the persistent kernel alone: every instance back in it
  if (merge_split(b) != hipSuccess) return AA_EHIP;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return AA_EHIP;
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // FNV-1a over the workload: variant, flags, every instance's (n, m, dim)
  uint64_t sig = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      sig ^= (v >> (8 * i)) & 0xffu;
      sig *= 1099511628211ull;
    }
  };
  mix(2u);  // cache format: grid, order, row pairs
  mix((uint64_t)b->variant);
  mix((uint64_t)b->flags);
  for (int j = 0; j < b->count; ++j) {
    mix((uint64_t)b->n[j]);
    mix((uint64_t)b->m[j]);
    mix((uint64_t)b->dim[j]);
  }
  char sigs[32];
  snprintf(sigs, sizeof sigs, "%016llx", (unsigned long long)sig);
  const bool graph = b->use_graph;
  if (cache_path) {
    // the last line matching this device and workload wins
    bool hit = false;
    aa_batch_schedule got{0, 0, 0.0, 0, 4};
    if (FILE* fh = fopen(cache_path, "r")) {
      char line[512], arch[128], s2[64];
      int g = 0, o = 0, pr = 0;
      double ms = 0.0;
      while (fgets(line, sizeof line, fh))
        if (sscanf(line, "%127s %63s %d %d %d %lf", arch, s2, &g, &o, &pr, &ms) == 6 &&
            strcmp(arch, prop.gcnArchName) == 0 && strcmp(s2, sigs) == 0 && g >= 0 && o >= 0 &&
            o <= 1 && (pr == 2 || pr == 4)) {
          hit = true;
          got = aa_batch_schedule{g, o, ms, 0, pr};
        }
      fclose(fh);
    }
    if (hit) {
      aa_status st = aa_batch_set_tiles(b, got.pairs);
      if (st == AA_OK) st = aa_batch_set_schedule(b, got.grid, got.order, graph);
      if (st != AA_OK) return st;
      if (best) *best = got;
      return AA_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return AA_EHIP;
  }
  aa_status st = AA_OK;
  aa_batch_schedule win{0, 0, 1e300, 0, 4};
  // tiles (row pairs per lane: 4 or 2) x persistent workgroups per compute
  // unit x instance order
  for (int pr = 4; pr >= 2 && st == AA_OK; pr -= 2) {
    b->pairs = pr;
    for (int per = 1; per <= 4 && st == AA_OK; ++per) {
      const int g = std::min(per * cus, b->count);
      if (per > 1 && g == std::min((per - 1) * cus, b->count)) break;  // capped: no new candidate
      for (int o = 0; o <= 1 && st == AA_OK; ++o) {
        st = aa_batch_set_schedule(b, g, o, 0);
        if (st != AA_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e0, b->stream) != hipSuccess || enqueue(b, iters) != hipSuccess ||
            hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = AA_EHIP;
          break;
        }
        win.trials += 1;
        if (ms / iters < win.ms_per_iter) {
          win.grid = g;
          win.order = o;
          win.pairs = pr;
          win.ms_per_iter = ms / iters;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AA_OK) return st;
  b->pairs = win.pairs;
  st = aa_batch_set_schedule(b, win.grid, win.order, graph);
  if (st != AA_OK) return st;
  if (cache_path) {
    if (FILE* fh = fopen(cache_path, "a")) {
      fprintf(fh, "%s %s %d %d %d %.6f\n", prop.gcnArchName, sigs, win.grid, win.order,
              win.pairs, win.ms_per_iter);
      fclose(fh);
    }
  }
  if (best) *best = win;
  return AA_OK;
}

aa_status aa_batch_run(aa_batch* b, int iters) {
  if (!b || iters < 0) return AA_EINVAL;
  if (iters == 0) return AA_OK;
  if (b->split_min_n > 0) {
    const aa_status s = update_split(b);
    if (s != AA_OK) return s;
  }
  if (!b->split.empty()) {
    // the persistent kernel leaves the split instances out; each of them
    // then runs its iteration on the grid-wide passes (host sequenced)
    for (int i = 0; i < iters; ++i) {
      if (enqueue_mode(b, BM_PLAIN, 0.f) != hipSuccess) return AA_EHIP;
      if (enqueue_split(b) != hipSuccess) return AA_EHIP;
    }
    return AA_OK;
  }
  if (!b->use_graph || b->stream == nullptr) return enqueue(b, iters) == hipSuccess ? AA_OK : AA_EHIP;
  if (b->exec_iters != iters) {
    drop_graph(b);
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return AA_EHIP;
    hipError_t e = enqueue(b, iters);
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return AA_EHIP;
    }
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return AA_EHIP;
    }
    b->exec_iters = iters;
  }
  return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? AA_OK : AA_EHIP;
}

aa_status aa_batch_read(aa_batch* b, aa_batch_state* states, int* active) {
  if (!b) return AA_EINVAL;
  std::vector<BState> hs(b->count);
  if (hipMemcpyAsync(hs.data(), b->d_state, sizeof(BState) * b->count, hipMemcpyDeviceToHost,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return AA_EHIP;
  if (states) memcpy(states, hs.data(), sizeof(BState) * b->count);
  if (active) {
    int a = 0;
    for (const BState& st : hs) a += st.active ? 1 : 0;
    *active = a;
  }
  return AA_OK;
}

aa_status aa_batch_run_learned(aa_batch* b, aa_mlp* net, int iters) {
  if (!b || !net || iters < 0 || !b->learned) return AA_EINVAL;
  if (mlp_stream(net) != b->stream || mlp_max_batch(net) < b->count) return AA_EINVAL;
  if (merge_split(b) != hipSuccess) return AA_EHIP;  // the learned step is one-workgroup only
  for (int i = 0; i < iters; ++i) {
    if (enqueue_mode(b, BM_PHASE_A, 0.f) != hipSuccess) return AA_EHIP;
    aa_status s = aa_mlp_forward(net, b->count, b->d_feat, b->d_out);
    if (s != AA_OK) return s;
    if (enqueue_mode(b, BM_GUARD, 0.f) != hipSuccess) return AA_EHIP;
  }
  return AA_OK;
}

aa_status aa_batch_train(aa_batch* b, aa_mlp* net, int iters, float lr) {
  if (!b || !net || iters < 0 || !b->learned || !(lr >= 0.f)) return AA_EINVAL;
  if (mlp_stream(net) != b->stream || mlp_max_batch(net) < b->count) return AA_EINVAL;
  if (merge_split(b) != hipSuccess) return AA_EHIP;
  const float dscale = 1.0f / (float)b->count;
  for (int i = 0; i < iters; ++i) {
    if (enqueue_mode(b, BM_PHASE_A, 0.f) != hipSuccess) return AA_EHIP;
    aa_status s = aa_mlp_forward(net, b->count, b->d_feat, b->d_out);
    if (s != AA_OK) return s;
    if (enqueue_mode(b, BM_TRAIN, dscale) != hipSuccess) return AA_EHIP;
    s = aa_mlp_backward(net, b->count, b->d_dout);
    if (s != AA_OK) return s;
    s = aa_mlp_adam(net, lr, 0.9f, 0.999f, 1e-8f);
    if (s != AA_OK) return s;
  }
  return AA_OK;
}

aa_status aa_batch_read_learning(aa_batch* b, float* feat, float* out, float* dout) {
  if (!b || !b->learned) return AA_EINVAL;
  const size_t c = (size_t)b->count;
  if ((feat && hipMemcpyAsync(feat, b->d_feat, sizeof(float) * c * kFeat, hipMemcpyDeviceToHost,
                              b->stream) != hipSuccess) ||
      (out && hipMemcpyAsync(out, b->d_out, sizeof(float) * c * kOuts, hipMemcpyDeviceToHost,
                             b->stream) != hipSuccess) ||
      (dout && hipMemcpyAsync(dout, b->d_dout, sizeof(float) * c * kOuts, hipMemcpyDeviceToHost,
                              b->stream) != hipSuccess) ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return AA_EHIP;
  return AA_OK;
}

aa_status aa_batch_destroy(aa_batch* b) {
  if (!b) return AA_OK;
  drop_graph(b);
  for (aa_ctx* v : b->views) view_destroy(v);
  delete b;
  return AA_OK;
}

}  // extern "C"
