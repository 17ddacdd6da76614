// aa_kernels.hip -- grid-wide FP64 HIP kernels for gfx950 of the windowed-QR
// Anderson acceleration update (Lockhart et al., arXiv 2110.09667, Algs. 1-6).
//
// Every kernel streams the tall-skinny n x k basis Q (column-major, padded
// leading dimension) from HBM once per pass.  A "Sync" of the paper -- a
// global reduction -- is one pass kernel: each workgroup folds its tiles into
// per-wave partial sums in LDS and publishes one partial per reduced value;
// a one-workgroup finalize kernel then sums the partials in a fixed order and
// runs the small dense tail on the device (R and T updates, the T solve of
// ICWY, the back substitution for gamma).  Results are bitwise reproducible
// for a given grid, and no value crosses to the host.  The pass bodies live in
// aa_passes.h (shared with the workgroup-level batched step).
#include <math.h>

#include <mutex>

#include "aa_passes.h"

namespace aa {

// Combine the per-wave accumulators of this workgroup and publish them as this
// workgroup's entries of the partials ([value][workgroup]); k_finalize, the
// next kernel on the stream, reduces them (the kernel boundary orders the
// writes before the reads, so no fence or atomic is needed here).
__device__ void publish(const Small& sm, int nred, const double* acc, int acc_stride) {
  __syncthreads();
  const int G = gridDim.x, b = blockIdx.x;
  for (int c = threadIdx.x; c < nred; c += kWG) {
    double s = acc[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += acc[w * acc_stride + c];
    sm.partials[(size_t)c * G + b] = s;
  }
}

// Sum of the G partials of one value by one wave: lane l adds partials
// l, l + 64, ... into eight interleaved accumulators (eight independent loads
// in flight per lane), combined in a fixed tree, then across the lanes.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int G, int lane) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int g = lane;
  for (; g + 7 * 64 < G; g += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[g + u * 64];
  }
  for (int u = 0; g < G; g += 64, ++u) a[u & 7] += p[g];
  const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return wave_sum(s);
}

// Fixed-order sum of the G partials of each of the nred values (one wave per
// value, two values per wave in flight), then the dense tail.
// Sums of the G partials of each value, one wave per value in the same fixed
// order as k_finalize's (bitwise the same sums), stored after the partials
// at partials[nred * G + c].  For the wide ICWY Gram (over a thousand values
// from hundreds of workgroups: 6.9 MB at m = 50) one workgroup reading them
// alone took 156 us.
__global__ __launch_bounds__(kWG) void k_sum_partials(Small sm, int nred, int G) {
  if (aa_stopped(sm)) return;
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (c >= nred) return;
  const double s = sum_partials(sm.partials + (size_t)c * G, G, lane);
  if (lane == 0) sm.partials[(size_t)nred * G + c] = s;
}

// pre: the sums were formed by k_sum_partials.
__global__ __launch_bounds__(kFinWG) void k_finalize(Small sm, Tail t, int nred, int G, int pre) {
  __shared__ double red[kMaxRedAll];
  if (sm.stop) {
    // the x update's finalize ends an iteration that broke down (its x update
    // wrote G(x_i)); the iteration counter already names the next one
    if (t.op == TAIL_STEP && threadIdx.x == 0 && sm.stop->done == 0 && *sm.status != AA_OK) {
      sm.stop->iter = sm.stop->cur - 1;
      sm.stop->k = t.k;
      sm.stop->m_i = t.m_i;
      sm.stop->done = AA_STOPPED_BREAKDOWN;
    }
    if (aa_stopped(sm)) return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int waves = kFinWG / 64;
  if (pre) {
    for (int c = threadIdx.x; c < nred; c += kFinWG) red[c] = sm.partials[(size_t)nred * G + c];
  } else {
    for (int c = w; c < nred; c += 2 * waves) {
      const int c2 = c + waves;
      const double s1 = sum_partials(sm.partials + (size_t)c * G, G, lane);
      const double s2 = c2 < nred ? sum_partials(sm.partials + (size_t)c2 * G, G, lane) : 0.0;
      if (lane == 0) {
        red[c] = s1;
        if (c2 < nred) red[c2] = s2;
      }
    }
  }
  __syncthreads();
  if (t.op != TAIL_GRAM_ADD) {
    run_tail(sm, t, red);
    return;
  }
  // QRDelete fused with the QRAdd's first pass: red holds the Gram pairs of
  // [q_0 .. q_{k-1}, v, (f)] (pair a(a-1)/2 + b, b < a).  Refresh T (ICWY),
  // then lay out what the first pass would have reduced -- Q^T v, the Gram
  // row of q_{k-1} where the variant uses it, Q^T f -- and run its tail.
  __shared__ double red2[kMaxRed];
  const int k = t.k;
  if (t.gram_t) {
    Tail tg = t;
    tg.op = TAIL_GRAM;
    run_tail(sm, tg, red);
  }
  const int pv = k * (k - 1) / 2, pf = (k + 1) * k / 2, prow = (k - 1) * (k - 2) / 2;
  const bool row = t.inner == TAIL_ICWY || (t.inner == TAIL_DCGS2 && t.reorth);
  for (int b = threadIdx.x; b < k; b += kFinWG) {
    red2[b] = red[pv + b];
    if (row && b < k - 1) red2[k + b] = red[prow + b];
    if (t.rhs) red2[t.zoff + b] = red[pf + b];
  }
  __syncthreads();
  Tail ti = t;
  ti.op = t.inner;
  run_tail(sm, ti, red2);
}

__global__ __launch_bounds__(kWG) void k_dots(DotsArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  __shared__ double s_acc[kWaves * kMaxRed];
  lds_zero(s_acc, kWaves * kMaxRed);
  __syncthreads();
  dots_body(a, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6) * kMaxRed);
  publish(sm, dots_nred(a), s_acc, kMaxRed);
}

// Block dot products with per-lane register accumulators (dots_reg_body):
// KQ-column buckets, one to three right-hand sides.
#ifndef AA_DOTS_REG
#define AA_DOTS_REG 1
#endif
#ifndef AA_DOTS_REG3
#define AA_DOTS_REG3 AA_DOTS_REG
#endif
template <int KQ, int NR>
__global__ __launch_bounds__(kWG) void k_dots_reg(DotsArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  constexpr int STR = NR * KQ + 2;  // nx + ny + nz + xx + xz <= NR KQ + 2
  __shared__ double s_acc[kWaves * STR];
  lds_zero(s_acc, kWaves * STR);
  __syncthreads();
  dots_reg_body<KQ, NR>(a, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6) * STR);
  publish(sm, dots_nred(a), s_acc, STR);
}

__global__ __launch_bounds__(kWG) void k_update(UpdArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  __shared__ double s_c1[kMaxCols], s_c2[kMaxCols], s_s[kMaxCols];
  __shared__ double s_acc[kWaves * 4];
  update_coefs(a, s_c1, s_c2, s_s);
  lds_zero(s_acc, kWaves * 4);
  __syncthreads();
  update_body(a, s_c1, s_c2, s_s, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6) * 4);
  publish(sm, update_nred(a), s_acc, 4);
}

// Column buckets up to AA_CGS2B_PAIR_MAX take the row-pair form (32: the
// 32-column bucket too, with one pair per lane).
#ifndef AA_CGS2B_PAIR_MAX
#define AA_CGS2B_PAIR_MAX 32
#endif
template <int KMAX>
__global__ __launch_bounds__(kWG) void k_cgs2b(Cgs2bArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  __shared__ double s_s[KMAX];
  __shared__ double s_acc[kWaves * KMAX];
  for (int j = threadIdx.x; j < KMAX; j += kWG) s_s[j] = (j < a.k) ? a.s[j] : 0.0;
  lds_zero(s_acc, kWaves * KMAX);
  __syncthreads();
  if constexpr (KMAX <= AA_CGS2B_PAIR_MAX)
    cgs2b_pair_body<KMAX, (KMAX <= 16 ? kPairs : 1)>(a, s_s, blockIdx.x, gridDim.x,
                                                     s_acc + (threadIdx.x >> 6) * KMAX);
  else
    cgs2b_body<KMAX>(a, s_s, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6) * KMAX);
  publish(sm, a.k, s_acc, KMAX);
}

__global__ __launch_bounds__(64) void k_givens(Small sm, int k, int transform) {
  if (aa_stopped(sm)) return;
  __shared__ double H[kMaxCols * kMaxCols];
  givens_body(sm, k, H);
  if (transform) {
    __syncthreads();  // H is free once R is written: it holds the Gram matrix
    t_transform_body(sm, k, H);
  }
}

template <int CH>
__global__ __launch_bounds__(kWG) void k_rotate(RotArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  __shared__ double s_c[kMaxCols], s_s[kMaxCols];
  givens_coefs(a, sm.cap, s_c, s_s, kMaxCols);
  __syncthreads();
  rotate_body<CH>(a, s_c, s_s, blockIdx.x, gridDim.x);
}

// Load depth of the plain rotation for long columns (n >= AA_ROT_LONG_N): at
// n = 2^25 and 2^26 four column pairs in flight per lane streamed 5-9 %
// faster than eight for k >= 19 (about the same at k = 9); at n = 2^24 eight
// were faster at k = 19.
#ifndef AA_ROT_LONG_N
#define AA_ROT_LONG_N (1ll << 25)
#endif
#ifndef AA_ROT_CH_LONG
#define AA_ROT_CH_LONG 4
#endif

// WAVES waves per workgroup: wide Gram staging (KMAX = 64 needs 25 KiB per
// wave) uses two-wave workgroups so that three of them share a compute unit
// (six waves) instead of one four-wave workgroup.
// Load depth of the rotation in the 64-column kernel: its staging leaves at
// most six waves per compute unit, so each lane keeps this many column loads
// in flight (measured at n = 2^26, k = 63: 30.2 ms with 8, 26.5 with 16,
// 25.4 with 32).
#ifndef AA_ROT_CH_WIDE
#define AA_ROT_CH_WIDE 32
#endif
constexpr int kRotChWide = AA_ROT_CH_WIDE;
// Load depth in the 16- and 32-column kernels.
#ifndef AA_ROT_CH_MID
#define AA_ROT_CH_MID 8
#endif
constexpr int kRotChMid = AA_ROT_CH_MID;

template <int KMAX, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_rotate_gram(RotArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  // staging rows, then the per-wave pair sums: gram_lds_doubles(gram_cols(a), WAVES)
  extern __shared__ double s_buf[];
  __shared__ double s_c[KMAX], s_s[KMAX];
  const int na = gram_cols(a), np = na * (na - 1) / 2;
  givens_coefs(a, sm.cap, s_c, s_s, KMAX);
  __syncthreads();
  v4d acc[GramShape<KMAX>::NBP];
  rotate_gram_body<KMAX, 64 * WAVES, (KMAX >= 64 ? kRotChWide : kRotChMid)>(
      a, s_c, s_s, blockIdx.x, gridDim.x, s_buf, gram_stride(na), acc);
  __syncthreads();  // the staging area becomes the per-wave pair accumulators
  gram_store<KMAX>(acc, s_buf + (threadIdx.x >> 6) * np, na);
  __syncthreads();
  const int G = gridDim.x, b = blockIdx.x;
  for (int c = threadIdx.x; c < np; c += 64 * WAVES) {
    double s = s_buf[c];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) s += s_buf[w * np + c];
    sm.partials[(size_t)c * G + b] = s;
  }
}

// 33 to 64 staged columns with the half-width staging (rotate_gram_split_body):
// four-wave workgroups, 64 x 33 doubles of LDS per wave, later reused for the
// per-wave pair sums.
#ifndef AA_ROT_CH_SPLIT
#define AA_ROT_CH_SPLIT 8
#endif
constexpr int kRotChSplit = AA_ROT_CH_SPLIT;
// The two-wave 64-column kernel stages 64 x gram_stride(na) doubles per wave:
// up to na = 53 three of its workgroups (six waves) share a compute unit's
// 160 KiB, beyond that only two (four waves, one per SIMD, so the MFMA phase
// of a tile cannot overlap another wave's loads).  From na = 54 on the
// half-staging kernel (eight waves) is faster: at n = 2^26, 63 columns,
// 17.5 ms instead of 25.5; at 48-49 columns it is 10-17 % slower.
#ifndef AA_GRAM_SPLIT_MIN
#define AA_GRAM_SPLIT_MIN 54
#endif
constexpr int kGramSplitMin = AA_GRAM_SPLIT_MIN;

__host__ __device__ constexpr int gram_split_lds_doubles(int na) {
  return kWaves * 64 * kHalfStride > kWaves * (na * (na - 1) / 2)
             ? kWaves * 64 * kHalfStride
             : kWaves * (na * (na - 1) / 2);
}

__global__ __launch_bounds__(kWG) void k_rotate_gram_split(RotArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  extern __shared__ double s_buf[];
  __shared__ double s_c[64], s_s[64];
  const int na = gram_cols(a), np = na * (na - 1) / 2;
  givens_coefs(a, sm.cap, s_c, s_s, 64);
  __syncthreads();
  v4d acc[10];
  rotate_gram_split_body<kWG, kRotChSplit>(a, s_c, s_s, blockIdx.x, gridDim.x, s_buf, acc);
  __syncthreads();  // the staging area becomes the per-wave pair accumulators
  gram_store<64>(acc, s_buf + (threadIdx.x >> 6) * np, na);
  publish(sm, np, s_buf, np);
}

// ICWY QRDelete for at most NAMAX (4 or 8) staged columns: rotation and strict
// lower Gram on the vector units (rotate_gram_small_body), per-wave pair sums
// by one butterfly reduction, then the usual per-workgroup partials.
constexpr int kGramSmall = 8;

template <int NAMAX>
__global__ __launch_bounds__(kWG) void k_rotate_gram_small(RotArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  constexpr int NR = NAMAX == 4 ? 8 : 32;  // NAMAX (NAMAX - 1) / 2 pairs, padded
  __shared__ double s_c[NAMAX], s_s[NAMAX];
  __shared__ double s_acc[kWaves * NR];
  const int na = gram_cols(a), np = na * (na - 1) / 2;
  givens_coefs(a, sm.cap, s_c, s_s, NAMAX);
  __syncthreads();
  double acc[NR];
  rotate_gram_small_body<NAMAX>(a, s_c, s_s, blockIdx.x, gridDim.x, acc);
  const double r = multi_reduce<NR>(acc);
  const int lane = threadIdx.x & 63;
  if (lane < NR) s_acc[(threadIdx.x >> 6) * NR + lane] = r;
  publish(sm, np, s_acc, NR);
}

__global__ __launch_bounds__(kWG) void k_scale(ScaleArgs a) {
  if (a.stop && (a.stop->done != 0 || *a.status != AA_OK)) return;
  scale_body(a.in, a.out, a.n, a.R[a.kk + (size_t)a.kk * a.cap], blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kWG) void k_history(HistArgs a, Small sm) {
  if (aa_stopped(sm)) return;
  __shared__ double s_acc[kWaves * 2];
  lds_zero(s_acc, kWaves * 2);
  __syncthreads();
  history_body(a, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6) * 2);
  publish(sm, a.first ? 2 : 1, s_acc, 2);
}

__global__ __launch_bounds__(kWG) void k_xupdate(XupdArgs a, Small sm) {
  if (aa_stopped(sm)) {
    // the iteration has ended: x_next = x, except in the step that broke down
    // (breakdown latched, not yet recorded as the end), which returns G(x_i)
    const double* src = sm.stop->done == 0 ? a.g : a.x;
    if (a.x_next != src)
      for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < a.n;
           r += (int64_t)gridDim.x * kWG)
        a.x_next[r] = src[r];
    return;
  }
  __shared__ double s_g[kMaxCols];
  __shared__ int s_slot[kMaxCols];
  __shared__ double s_acc[kWaves];
  xupdate_coefs(a, s_g, s_slot);
  lds_zero(s_acc, kWaves);
  __syncthreads();
  xupdate_body(a, s_g, s_slot, blockIdx.x, gridDim.x, s_acc + (threadIdx.x >> 6));
  publish(sm, 1, s_acc, 1);
}

// The batched state of an instance advanced on the grid-wide passes: its
// next iteration, columns, window and residual while it runs; its stopping
// iteration once its stop state has ended it (the batch's convention: the
// iteration at whose start the test held is not counted as run).  G
// evaluations: G(x_0) plus one per iteration begun.
__global__ void k_split_state(BState* st, const StopState* stop, const double* scal,
                              const int* status, int k, int m_i) {
  if (threadIdx.x != 0) return;
  BState s = *st;
  s.res_norm = sqrt(scal[S_RES]);
  s.status = *status;
  if (stop->done) {
    s.active = 0;
    s.iter = stop->iter;
    if (s.conv_iter < 0) s.conv_iter = stop->iter;
    s.k = stop->k;
    s.m_i = stop->m_i;
    s.g_evals = stop->iter + 1;
  } else {
    s.iter = stop->cur;
    s.k = k;
    s.m_i = m_i;
    s.g_evals = stop->cur;
  }
  *st = s;
}

__global__ void k_set_int(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_set_int(int* p, int64_t n, int v, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 1024 ? blocks : 1024);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_set_int, dim3(grid), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_split_state(BState* st, const StopState* stop, const Small& sm, int k, int m_i,
                              hipStream_t s) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_split_state, dim3(1), dim3(64), 0, s, st, stop, sm.scal, sm.status, k,
                     m_i);
  return hipGetLastError();
}

// Ends the iteration at the cap of aa_set_stop (if nothing ended it before)
// and writes x_next = x.
__global__ __launch_bounds__(kWG) void k_stop_cap(StopState* stop, int k, int m_i,
                                                  const double* x, double* xn, int64_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && stop->done == 0) {
    stop->iter = stop->cur;
    stop->k = k;
    stop->m_i = m_i;
    stop->done = AA_STOPPED_CAP;
  }
  if (xn != x)
    for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < n; r += (int64_t)gridDim.x * kWG)
      xn[r] = x[r];
}

__global__ void k_init_small(Small sm) {
  const int cap = sm.cap;
  const int64_t tot = (int64_t)cap * cap;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    sm.R[i] = 0.0;
    sm.T[i] = ((i % cap) == (i / cap)) ? 1.0 : 0.0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * cap; i += gridDim.x * blockDim.x)
    sm.givens[i] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
    sm.coef0[i] = 0.0;
    sm.coef1[i] = 0.0;
    sm.gamma[i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x < S_COUNT) sm.scal[threadIdx.x] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *sm.status = AA_OK;
    if (sm.stop) {
      sm.stop->done = 0;
      sm.stop->k = 0;
      sm.stop->m_i = 0;
      sm.stop->iter = 0;
      sm.stop->cur = 0;
    }
  }
}

__global__ void k_copy(double* dst, const double* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Bandwidth probe with the passes' access pattern (same tiles, 16-byte
// non-temporal loads of full tiles, plain stores as in the update pass):
// read RD vectors of length n (leading dimension ld), write WR vectors, each
// written vector the sum of the read ones; with no write, each workgroup
// writes one partial sum to sink so the loads cannot be dropped.
template <int RD, int WR>
__global__ __launch_bounds__(kWG) void k_probe(const double* src, int64_t ld, double* dst,
                                               int64_t n, double* sink) {
  double acc = 0.0;
  for_tiles(n, blockIdx.x, gridDim.x, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 v[RD][kPairs];
#pragma unroll
    for (int j = 0; j < RD; ++j) ld2<F>(v[j], src + (int64_t)j * ld, b2, n);
    double2 o[kPairs];
    zero2(o);
#pragma unroll
    for (int j = 0; j < RD; ++j)
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        o[i].x += v[j][i].x;
        o[i].y += v[j][i].y;
      }
    if constexpr (WR > 0) {
#pragma unroll
      for (int w = 0; w < WR; ++w) st2<F>(o, dst + (int64_t)w * ld, b2, n);
    } else {
#pragma unroll
      for (int i = 0; i < kPairs; ++i) acc += o[i].x + o[i].y;
    }
  });
  if constexpr (WR == 0) {
    __shared__ double s_w[kWaves];
    const double t = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double u = 0.0;
      for (int w = 0; w < kWaves; ++w) u += s_w[w];
      sink[blockIdx.x] = u;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {
thread_local hipEvent_t t_prof_mid = nullptr;
thread_local bool t_prof_mid_used = false;
}  // namespace

void set_profile_mid(hipEvent_t e) {
  t_prof_mid = e;
  t_prof_mid_used = false;
}

bool profile_mid_used() { return t_prof_mid_used; }

// Workgroups of `kernel` (threads, dynamic LDS) that the device holds at once;
// 0 if unknown.  A grid-stride pass launched with more workgroups than that
// (but fewer than twice as many) runs its last round on part of the chip: the
// Gram kernels hold 2-4 workgroups per compute unit, some dot-product
// instances 3.  Answers are cached per (device, kernel, threads, LDS).
static int resident_workgroups(const void* kernel, int threads, size_t lds) {
  struct Entry { const void* k; int threads; size_t lds; int dev; int res; };
  static Entry cache[128];
  static int used = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  {
    std::lock_guard<std::mutex> g(mu);
    for (int i = 0; i < used; ++i)
      if (cache[i].k == kernel && cache[i].threads == threads && cache[i].lds == lds &&
          cache[i].dev == dev)
        return cache[i].res;
  }
  int cus = 0, per_cu = 0;
  const bool ok =
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();  // a failed query must not be reported by the launch
    return 0;
  }
  const int res = per_cu * cus;
  std::lock_guard<std::mutex> g(mu);
  if (used < 128) cache[used++] = Entry{kernel, threads, lds, dev, res};
  return res;
}

static int clamp_resident(int grid, const void* kernel, int threads, size_t lds) {
  const int r = resident_workgroups(kernel, threads, lds);
  return (r > 0 && grid > r) ? r : grid;
}

// Partials (values x workgroups) from which the sums run on one wave per
// value before the finalize.
#ifndef AA_SUM_PARTIALS_MIN
#define AA_SUM_PARTIALS_MIN 65536
#endif
constexpr int64_t kSumPartialsMin = AA_SUM_PARTIALS_MIN;

static hipError_t launch_finalize(const Small& sm, const Tail& t, int nred, int grid,
                                  hipStream_t st) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (t_prof_mid) {
    e = hipEventRecord(t_prof_mid, st);
    if (e != hipSuccess) return e;
    t_prof_mid_used = true;
  }
  // many partials (the wide Gram): sum them with one wave per value first
  const int64_t many = (int64_t)nred * grid;
  const int pre = many >= kSumPartialsMin && sm.npart >= many + nred ? 1 : 0;
  if (pre)
    hipLaunchKernelGGL(k_sum_partials, dim3((nred + kWaves - 1) / kWaves), dim3(kWG), 0, st, sm,
                       nred, grid);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinWG), 0, st, sm, t, nred, grid, pre);
  return hipGetLastError();
}

hipError_t launch_dots(const DotsArgs& a, const Small& sm, const Tail& t, int grid,
                       hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  // every vector the counts name must exist
  if (!a.x || (a.ny > 0 && !a.y) || (a.nz > 0 && !a.z) || (a.xz && a.nz < 1))
    return hipErrorInvalidValue;
  // one round of resident workgroups at most; the finalize sums `grid` partials
  auto clamp_launch = [&](const void* kern, auto launch) {
    const int g = clamp_resident(grid, kern, kWG, 0);
    launch(g);
    return g;
  };
  int nq = a.nx > a.ny ? a.nx : a.ny;
  if (a.nz > nq) nq = a.nz;
  const int nr = a.nz > 0 ? 3 : (a.ny > 0 ? 2 : 1);  // right-hand sides
  if (AA_DOTS_REG && nr == 1 && nq <= 8)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<8, 1>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<8, 1>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 1 && nq <= 16)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<16, 1>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<16, 1>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 1 && nq <= 32)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<32, 1>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<32, 1>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 1 && nq <= 64)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<64, 1>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<64, 1>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 2 && nq <= 8)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<8, 2>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<8, 2>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 2 && nq <= 16)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<16, 2>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<16, 2>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG && nr == 2 && nq <= 32)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<32, 2>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<32, 2>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG3 && nr == 3 && nq <= 8)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<8, 3>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<8, 3>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG3 && nr == 3 && nq <= 16)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<16, 3>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<16, 3>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else if (AA_DOTS_REG3 && nr == 3 && nq <= 32)
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots_reg<32, 3>), [&](int g) {
      hipLaunchKernelGGL((k_dots_reg<32, 3>), dim3(g), dim3(kWG), 0, st, a, sm);
    });
  else
    grid = clamp_launch(reinterpret_cast<const void*>(&k_dots), [&](int g) {
      hipLaunchKernelGGL(k_dots, dim3(g), dim3(kWG), 0, st, a, sm);
    });
  return launch_finalize(sm, t, a.nx + a.ny + a.nz + (a.xx ? 1 : 0) + (a.xz ? 1 : 0), grid, st);
}

hipError_t launch_update(const UpdArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  grid = clamp_resident(grid, reinterpret_cast<const void*>(&k_update), kWG, 0);
  hipLaunchKernelGGL(k_update, dim3(grid), dim3(kWG), 0, st, a, sm);
  if (update_nred(a) == 0) return hipGetLastError();  // nothing reduced: no Sync
  return launch_finalize(sm, t, update_nred(a), grid, st);
}

hipError_t launch_cgs2b(const Cgs2bArgs& a, const Small& sm, const Tail& t, int grid,
                        hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  auto go = [&](const void* kern, auto launch) {
    grid = clamp_resident(grid, kern, kWG, 0);
    launch();
  };
  if (a.k <= 8) {
    go(reinterpret_cast<const void*>(&k_cgs2b<8>),
       [&] { hipLaunchKernelGGL(k_cgs2b<8>, dim3(grid), dim3(kWG), 0, st, a, sm); });
  } else if (a.k <= 16) {
    go(reinterpret_cast<const void*>(&k_cgs2b<16>),
       [&] { hipLaunchKernelGGL(k_cgs2b<16>, dim3(grid), dim3(kWG), 0, st, a, sm); });
  } else if (a.k <= 32) {
    go(reinterpret_cast<const void*>(&k_cgs2b<32>),
       [&] { hipLaunchKernelGGL(k_cgs2b<32>, dim3(grid), dim3(kWG), 0, st, a, sm); });
  } else {
    go(reinterpret_cast<const void*>(&k_cgs2b<64>),
       [&] { hipLaunchKernelGGL(k_cgs2b<64>, dim3(grid), dim3(kWG), 0, st, a, sm); });
  }
  return launch_finalize(sm, t, a.k, grid, st);
}

hipError_t launch_givens(const Small& sm, int k, hipStream_t st, bool transform) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, sm, k, transform ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rotate(const RotArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  if (a.gram) {
    // The kernel instance must hold every rotated column (its Givens
    // coefficient arrays) and every staged one: w = max(k - 1, Gram columns).
    // The Gram's own column count na sizes the dynamic LDS (fewer columns,
    // more resident workgroups) and picks the 64-column variant.
    const int na = gram_cols(a), w = a.k - 1 + a.naug;
    // one round of resident workgroups at most (the finalize sums `grid`
    // partials per value)
    auto go = [&](const void* kern, int threads, size_t lds, auto launch) {
      grid = clamp_resident(grid, kern, threads, lds);
      launch(grid, threads, lds);
    };
    if (w <= 4) {
      go(reinterpret_cast<const void*>(&k_rotate_gram_small<4>), kWG, 0, [&](int g, int th, size_t l) {
        hipLaunchKernelGGL(k_rotate_gram_small<4>, dim3(g), dim3(th), l, st, a, sm);
      });
    } else if (w <= kGramSmall) {
      go(reinterpret_cast<const void*>(&k_rotate_gram_small<kGramSmall>), kWG, 0,
         [&](int g, int th, size_t l) {
           hipLaunchKernelGGL(k_rotate_gram_small<kGramSmall>, dim3(g), dim3(th), l, st, a, sm);
         });
    } else if (w <= 16) {
      go(reinterpret_cast<const void*>(&k_rotate_gram<16, kWaves>), kWG,
         sizeof(double) * (size_t)gram_lds_doubles(na, kWaves), [&](int g, int th, size_t l) {
           hipLaunchKernelGGL((k_rotate_gram<16, kWaves>), dim3(g), dim3(th), l, st, a, sm);
         });
    } else if (w <= 32) {
      go(reinterpret_cast<const void*>(&k_rotate_gram<32, kWaves>), kWG,
         sizeof(double) * (size_t)gram_lds_doubles(na, kWaves), [&](int g, int th, size_t l) {
           hipLaunchKernelGGL((k_rotate_gram<32, kWaves>), dim3(g), dim3(th), l, st, a, sm);
         });
    } else if (w <= 64 && na < kGramSplitMin) {
      go(reinterpret_cast<const void*>(&k_rotate_gram<64, 2>), 128,
         sizeof(double) * (size_t)gram_lds_doubles(na, 2), [&](int g, int th, size_t l) {
           hipLaunchKernelGGL((k_rotate_gram<64, 2>), dim3(g), dim3(th), l, st, a, sm);
         });
    } else if (w <= 64) {  // na >= kGramSplitMin > 32, as the half staging needs
      go(reinterpret_cast<const void*>(&k_rotate_gram_split), kWG,
         sizeof(double) * (size_t)gram_split_lds_doubles(na), [&](int g, int th, size_t l) {
           hipLaunchKernelGGL(k_rotate_gram_split, dim3(g), dim3(th), l, st, a, sm);
         });
    } else {
      return hipErrorInvalidValue;  // at most 64 rotated or staged columns
    }
    return launch_finalize(sm, t, na * (na - 1) / 2, grid, st);
  }
  if (a.n >= AA_ROT_LONG_N)
    hipLaunchKernelGGL(k_rotate<AA_ROT_CH_LONG>, dim3(grid), dim3(kWG), 0, st, a, sm);
  else
    hipLaunchKernelGGL(k_rotate<kRotChPair>, dim3(grid), dim3(kWG), 0, st, a, sm);
  return hipGetLastError();
}

hipError_t launch_scale(const ScaleArgs& a, const Small& sm, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  (void)sm;
  int64_t blocks = (a.n / 2 + kWG - 1) / kWG;
  int grid = (int)(blocks < 4096 ? blocks : 4096);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_scale, dim3(grid), dim3(kWG), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_history(const HistArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  grid = clamp_resident(grid, reinterpret_cast<const void*>(&k_history), kWG, 0);
  hipLaunchKernelGGL(k_history, dim3(grid), dim3(kWG), 0, st, a, sm);
  return launch_finalize(sm, t, a.first ? 2 : 1, grid, st);
}

hipError_t launch_xupdate(const XupdArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  grid = clamp_resident(grid, reinterpret_cast<const void*>(&k_xupdate), kWG, 0);
  hipLaunchKernelGGL(k_xupdate, dim3(grid), dim3(kWG), 0, st, a, sm);
  return launch_finalize(sm, t, 1, grid, st);
}

hipError_t launch_probe(int reads, int writes, const double* src, int64_t ld, double* dst,
                        int64_t n, double* sink, int grid, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  auto go = [&](const void* kern, auto launch) {
    grid = clamp_resident(grid, kern, kWG, 0);
    launch(grid);
  };
#define AA_PROBE(RD, WR)                                                              \
  if (reads == RD && writes == WR) {                                                   \
    go(reinterpret_cast<const void*>(&k_probe<RD, WR>), [&](int g) {                   \
      hipLaunchKernelGGL((k_probe<RD, WR>), dim3(g), dim3(kWG), 0, st, src, ld, dst, n, sink); \
    });                                                                                \
    return hipGetLastError();                                                          \
  }
  AA_PROBE(1, 0)
  AA_PROBE(4, 0)
  AA_PROBE(8, 0)
  AA_PROBE(1, 1)
  AA_PROBE(2, 1)
  AA_PROBE(3, 1)
  AA_PROBE(8, 1)
  AA_PROBE(1, 2)
#undef AA_PROBE
  return hipErrorInvalidValue;
}

hipError_t launch_init_small(const Small& sm, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_init_small, dim3(8), dim3(kWG), 0, st, sm);
  return hipGetLastError();
}

hipError_t launch_stop_cap(StopState* stop, int k, int m_i, const double* x, double* xn,
                           int64_t n, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (n + kWG - 1) / kWG;
  int grid = (int)(blocks < 1024 ? blocks : 1024);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_stop_cap, dim3(grid), dim3(kWG), 0, st, stop, k, m_i, x, xn, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (n + kWG - 1) / kWG;
  int grid = (int)(blocks < 4096 ? blocks : 4096);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kWG), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace aa
