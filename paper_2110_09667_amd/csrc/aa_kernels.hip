// aa_kernels.hip -- FP64 HIP kernels for gfx950 of the windowed-QR Anderson
// acceleration update (Lockhart et al., arXiv 2110.09667, Algs. 1-6).
//
// Every kernel streams the tall-skinny n x k basis Q (column-major, padded
// leading dimension) from HBM once per pass.  A "Sync" of the paper -- a
// global reduction -- is one kernel: each workgroup folds its rows into
// per-wave partial sums in LDS, publishes one partial per reduced value, and
// the last workgroup to arrive (atomic ticket) sums the partials in a fixed
// order and runs the small dense tail on the device (R and T updates, the T
// solve of ICWY, the back substitution for gamma).  Results are therefore
// bitwise reproducible for a given grid, and no value crosses to the host.
#include <math.h>

#include "aa_internal.h"

namespace aa {

// ---------------------------------------------------------------------------
// wavefront reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum N per-lane values across the 64 lanes at once (N a power of two, <= 64).
// Butterfly with halving: at the step of offset h, a lane keeps the half of
// its values selected by lane bit h and adds its partner's copy of that half.
// After log2(N) steps lane l holds column (l mod N) summed over the lanes that
// share its low bits; the remaining xor steps finish the sum.  N - 1 +
// 6 - log2(N) shuffles instead of 6 N.
template <int H, int N>
__device__ __forceinline__ void halve_step(double (&v)[N], int lane) {
  if constexpr (H >= 1) {
    const bool upper = (lane & H) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = upper ? v[i + H] : v[i];
      const double send = upper ? v[i] : v[i + H];
      v[i] = keep + __shfl_xor(send, H, 64);
    }
    halve_step<H / 2, N>(v, lane);
  }
}

template <int N>
__device__ __forceinline__ double multi_reduce(double (&v)[N]) {
  const int lane = threadIdx.x & 63;
  halve_step<N / 2, N>(v, lane);
  double r = v[0];
#pragma unroll
  for (int o = N; o < 64; o <<= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// ---------------------------------------------------------------------------
// grid-wide reduction by the last-arriving workgroup, and the dense tails
// ---------------------------------------------------------------------------

// Publish this workgroup's nred values; return true in the last workgroup.
__device__ bool arrive(const Small& sm, int nred, const double* wg_vals) {
  const int G = gridDim.x, b = blockIdx.x;
  for (int c = threadIdx.x; c < nred; c += kWG) sm.partials[(size_t)c * G + b] = wg_vals[c];
  __threadfence();
  __syncthreads();
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(sm.ticket, 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (unsigned)(G - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  return true;
}

// Fixed-order sum of the partials into red[] (LDS), then reset the ticket.
__device__ void collect(const Small& sm, int nred, double* red) {
  const int G = gridDim.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = w; c < nred; c += kWaves) {
    const double* p = sm.partials + (size_t)c * G;
    double s = 0.0;
    for (int g = lane; g < G; g += 64) s += p[g];
    s = wave_sum(s);
    if (lane == 0) red[c] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(sm.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void run_tail(const Small& sm, const Tail& t, const double* red) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int cap = sm.cap;
  double* R = sm.R;
  double* T = sm.T;
  const int k = t.k;
  switch (t.op) {
    case TAIL_STORE:
      for (int i = tid; i < t.count; i += kWG) sm.coef0[i] = red[i];
      break;
    case TAIL_MGS_R:
      if (tid == 0) R[t.row + (size_t)k * cap] = red[0];
      break;
    case TAIL_NORM:
      if (tid == 0) {
        const double nv = sqrt(red[t.idx]);
        R[k + (size_t)k * cap] = nv;
        if (!(nv > 0.0) || !isfinite(nv)) *sm.status = AA_EBREAKDOWN;
      }
      break;
    case TAIL_CGS2_S:
      for (int i = tid; i < k; i += kWG) sm.coef0[i] = red[i];
      break;
    case TAIL_CGS2_Z:
      for (int i = tid; i < k; i += kWG) {
        sm.coef1[i] = red[i];
        R[i + (size_t)k * cap] = sm.coef0[i] + red[i];
      }
      break;
    case TAIL_ICWY:
      // Alg. 4: row k-1 of T is red[k + b] (b < k-1), diagonal 1; solve the
      // unit lower triangular T r' = r with r = red[0:k] (forward
      // substitution, one lane per row); r' is column k of R and the
      // coefficients of the update pass.
      for (int b = tid; b < k - 1; b += kWG) T[(k - 1) + (size_t)b * cap] = red[k + b];
      if (tid < 64) {
        double x = (lane < k) ? red[lane] : 0.0;
        for (int b = 0; b < k; ++b) {
          const double rb = __shfl(x, b, 64);
          if (lane > b && lane < k) {
            const double tab = (lane == k - 1) ? red[k + b] : T[lane + (size_t)b * cap];
            x -= tab * rb;
          }
        }
        if (lane < k) {
          R[lane + (size_t)k * cap] = x;
          sm.coef0[lane] = x;
        }
      }
      break;
    case TAIL_DCGS2:
      // Alg. 6: column k of R is Q^T v computed with the old q_{k-1}; with
      // reorthogonalization s = red[k:2k-1] corrects column k-1 of R so that
      // Q R = F_i keeps holding after q_{k-1} -= Q_{:,0:k-2} s.
      for (int i = tid; i < k; i += kWG) R[i + (size_t)k * cap] = red[i];
      if (t.reorth) {
        const int p = k - 1;
        const double scale = t.literal ? 1.0 : R[p + (size_t)p * cap];
        for (int i = tid; i < p; i += kWG) {
          const double s = red[k + i];
          sm.coef1[i] = s;
          R[i + (size_t)p * cap] += scale * s;
        }
      }
      break;
    case TAIL_RHS:
      // Alg. 2, last line: back substitution R gamma = c, c = Q^T f_i.
      if (tid < 64) {
        double x = (lane < k) ? red[lane] : 0.0;
        double gam = 0.0;
        for (int a = k - 1; a >= 0; --a) {
          const double ga = __shfl(x, a, 64) / R[a + (size_t)a * cap];
          if (lane < a) x -= R[lane + (size_t)a * cap] * ga;
          if (lane == a) gam = ga;
        }
        if (lane < k) sm.gamma[lane] = gam;
      }
      break;
    case TAIL_RES:
      if (tid == 0) sm.scal[S_RES] = red[0];
      break;
    case TAIL_FIRST:
      if (tid == 0) {
        sm.scal[S_RES] = red[0];
        sm.scal[S_RES0] = red[0];
        sm.scal[S_STEP] = red[1];
      }
      break;
    case TAIL_STEP:
      if (tid == 0) sm.scal[S_STEP] = red[0];
      break;
    case TAIL_GRAM: {
      // ICWY after QRDelete: T_ab = q_a^T q_b (b < a < k), pair a(a-1)/2 + b.
      for (int a = 1; a < k; ++a)
        for (int b = tid; b < a; b += kWG) T[a + (size_t)b * cap] = red[a * (a - 1) / 2 + b];
      break;
    }
    default:
      break;
  }
}

// Combine the per-wave accumulators of this workgroup, then reduce across the
// grid; the last workgroup runs the tail.
__device__ void finish(const Small& sm, const Tail& t, int nred, const double* acc,
                       int acc_stride, double* red) {
  __syncthreads();
  for (int c = threadIdx.x; c < nred; c += kWG) {
    double s = acc[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += acc[w * acc_stride + c];
    red[c] = s;
  }
  __syncthreads();
  if (!arrive(sm, nred, red)) return;
  collect(sm, nred, red);
  run_tail(sm, t, red);
}

// ---------------------------------------------------------------------------
// row loads for the streaming passes (kRPT rows per thread, stride kWG)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void load_rows(double (&r)[kRPT], const double* __restrict__ p,
                                          int64_t base, int64_t n, bool full) {
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    const int64_t row = base + (int64_t)i * kWG;
    r[i] = (full || row < n) ? p[row] : 0.0;
  }
}

__device__ __forceinline__ void store_rows(const double (&r)[kRPT], double* p, int64_t base,
                                           int64_t n, bool full) {
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    const int64_t row = base + (int64_t)i * kWG;
    if (full || row < n) p[row] = r[i];
  }
}

__device__ __forceinline__ double dot_rows(const double (&a)[kRPT], const double (&b)[kRPT]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kRPT; ++i) s = fma(a[i], b[i], s);
  return s;
}

// ---------------------------------------------------------------------------
// block dot products: red = [Q^T x, Q_{:,0:ny-1}^T y, x^T x]
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWG) void k_dots(DotsArgs a, Small sm, Tail t) {
  __shared__ double s_acc[kWaves * kMaxRed];
  __shared__ double s_red[kMaxRed];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nq = a.nx > a.ny ? a.nx : a.ny;
  const int nred = a.nx + a.ny + (a.xx ? 1 : 0);
  for (int c = threadIdx.x; c < kWaves * kMaxRed; c += kWG) s_acc[c] = 0.0;
  __syncthreads();
  double* acc = s_acc + w * kMaxRed;
  const int64_t ntiles = (a.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kTile + threadIdx.x;
    const bool full = (tile + 1) * kTile <= a.n;
    double xv[kRPT], yv[kRPT];
    load_rows(xv, a.x, base, a.n, full);
    if (a.ny > 0) load_rows(yv, a.y, base, a.n, full);
    if (a.xx) {
      const double p = wave_sum(dot_rows(xv, xv));
      if (lane == 0) acc[a.nx + a.ny] += p;
    }
    for (int j = 0; j < nq; ++j) {
      double qv[kRPT];
      load_rows(qv, a.Q + (int64_t)j * a.ldq, base, a.n, full);
      if (j < a.nx) {
        const double p = wave_sum(dot_rows(qv, xv));
        if (lane == 0) acc[j] += p;
      }
      if (j < a.ny) {
        const double p = wave_sum(dot_rows(qv, yv));
        if (lane == 0) acc[a.nx + j] += p;
      }
    }
  }
  finish(sm, t, nred, s_acc, kMaxRed, s_red);
}

// ---------------------------------------------------------------------------
// vector update out = v - Q c (+ fused dot / norm); DCGS-2 reorthogonalization
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWG) void k_update(UpdArgs a, Small sm, Tail t) {
  __shared__ double s_c1[kMaxCols], s_c2[kMaxCols], s_s[kMaxCols];
  __shared__ double s_acc[kWaves * 4];
  __shared__ double s_red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < kMaxCols; j += kWG) {
    s_c1[j] = (a.c1 && j < a.j0 + a.nc + 1) ? a.c1[j] : 0.0;
    s_c2[j] = (a.c2 && j < a.j0 + a.nc) ? a.c2[j] : 0.0;
    s_s[j] = (a.s && a.dcgs2_p >= 0 && j < a.dcgs2_p) ? a.s[j] : 0.0;
  }
  if (threadIdx.x < kWaves * 4) s_acc[threadIdx.x] = 0.0;
  __syncthreads();
  const int nred = (a.dotcol >= 0 ? 1 : 0) + (a.nrm ? 1 : 0);
  const int inorm = a.dotcol >= 0 ? 1 : 0;
  const int64_t ntiles = (a.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kTile + threadIdx.x;
    const bool full = (tile + 1) * kTile <= a.n;
    double o[kRPT], acc1[kRPT], acc2[kRPT];
    load_rows(o, a.v, base, a.n, full);
#pragma unroll
    for (int i = 0; i < kRPT; ++i) acc1[i] = acc2[i] = 0.0;
    if (a.dcgs2_p >= 0) {
      // Alg. 6: q'_p = q_p - Q_{:,0:p-1} s, then v - Q_{:,0:p-1} c - q'_p c_p
      const int p = a.dcgs2_p;
#pragma unroll 2
      for (int j = 0; j < p; ++j) {
        double qv[kRPT];
        load_rows(qv, a.Q + (int64_t)j * a.ldq, base, a.n, full);
        const double cj = s_c1[j], sj = s_s[j];
#pragma unroll
        for (int i = 0; i < kRPT; ++i) {
          acc1[i] = fma(qv[i], cj, acc1[i]);
          acc2[i] = fma(qv[i], sj, acc2[i]);
        }
      }
      double qp[kRPT];
      load_rows(qp, a.Q + (int64_t)p * a.ldq, base, a.n, full);
      if (a.reorth) {
#pragma unroll
        for (int i = 0; i < kRPT; ++i) qp[i] -= acc2[i];
        store_rows(qp, a.Qw + (int64_t)p * a.ldq, base, a.n, full);
      }
      const double cp = s_c1[p];
#pragma unroll
      for (int i = 0; i < kRPT; ++i) o[i] = (o[i] - acc1[i]) - qp[i] * cp;
    } else {
#pragma unroll 2
      for (int j = a.j0; j < a.j0 + a.nc; ++j) {
        double qv[kRPT];
        load_rows(qv, a.Q + (int64_t)j * a.ldq, base, a.n, full);
        const double cj = s_c1[j], zj = s_c2[j];
#pragma unroll
        for (int i = 0; i < kRPT; ++i) {
          acc1[i] = fma(qv[i], cj, acc1[i]);
          acc2[i] = fma(qv[i], zj, acc2[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < kRPT; ++i) o[i] = (o[i] - acc1[i]) - acc2[i];
    }
    if (a.out) store_rows(o, a.out, base, a.n, full);
    if (a.dotcol >= 0) {
      double qv[kRPT];
      load_rows(qv, a.Q + (int64_t)a.dotcol * a.ldq, base, a.n, full);
      const double p = wave_sum(dot_rows(qv, o));
      if (lane == 0) s_acc[w * 4 + 0] += p;
    }
    if (a.nrm) {
      const double p = wave_sum(dot_rows(o, o));
      if (lane == 0) s_acc[w * 4 + inorm] += p;
    }
  }
  finish(sm, t, nred, s_acc, 4, s_red);
}

// ---------------------------------------------------------------------------
// CGS-2 second pass (Alg. 5): y = v - Q s in registers, red[j] = q_j^T y.
// One row per thread, the row's k values of Q held in registers.
// ---------------------------------------------------------------------------

template <int KMAX>
__global__ __launch_bounds__(kWG) void k_cgs2b(Cgs2bArgs a, Small sm, Tail t) {
  __shared__ double s_s[KMAX];
  __shared__ double s_acc[kWaves * KMAX];
  __shared__ double s_red[KMAX];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < KMAX; j += kWG) s_s[j] = (j < a.k) ? a.s[j] : 0.0;
  for (int c = threadIdx.x; c < kWaves * KMAX; c += kWG) s_acc[c] = 0.0;
  __syncthreads();
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kWG + threadIdx.x;
    const bool valid = row < a.n;
    double q[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      q[j] = (j < a.k && valid) ? a.Q[(int64_t)j * a.ldq + row] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc = fma(q[j], s_s[j], acc);
    const double y = (valid ? a.v[row] : 0.0) - acc;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) q[j] *= y;
    const double r = multi_reduce<KMAX>(q);
    if (lane < KMAX) s_acc[w * KMAX + lane] += r;
  }
  finish(sm, t, a.k, s_acc, KMAX, s_red);
}

// ---------------------------------------------------------------------------
// QRDelete (Alg. 2): Givens rotations from R (one wave), then one sweep over Q
// ---------------------------------------------------------------------------

// H = R_{:,1:k-1}; rotation j zeroes H_{j+1,j}; R <- the (k-1)x(k-1) triangle.
__global__ __launch_bounds__(64) void k_givens(Small sm, int k) {
  __shared__ double H[kMaxCols * kMaxCols];  // H[i + j * k]
  const int lane = threadIdx.x;
  const int cap = sm.cap;
  const int nc = k - 1;
  for (int j = 0; j < nc; ++j)
    for (int i = lane; i < k; i += 64) H[i + j * k] = sm.R[i + (size_t)(j + 1) * cap];
  __syncthreads();
  for (int j = 0; j < nc; ++j) {
    const double x = H[j + j * k], y = H[(j + 1) + j * k];
    const double rho = hypot(x, y);
    const double c = rho > 0.0 ? x / rho : 1.0;
    const double s = rho > 0.0 ? y / rho : 0.0;
    __syncthreads();
    for (int col = j + lane; col < nc; col += 64) {
      const double hj = H[j + col * k], hj1 = H[(j + 1) + col * k];
      H[j + col * k] = c * hj + s * hj1;
      H[(j + 1) + col * k] = -s * hj + c * hj1;
    }
    if (lane == 0) {
      sm.givens[j] = c;
      sm.givens[cap + j] = s;
    }
    __syncthreads();
    if (lane == 0) H[(j + 1) + j * k] = 0.0;
    __syncthreads();
  }
  for (int j = 0; j < k; ++j)
    for (int i = lane; i < k; i += 64)
      sm.R[i + (size_t)j * cap] = (i < nc && j < nc && i <= j) ? H[i + j * k] : 0.0;
}

// Pair p of the strict lower triangle in row order: p = a(a-1)/2 + b, b < a.
constexpr int pair_a(int p) {
  int a = 1;
  while ((a + 1) * a / 2 <= p) ++a;
  return a;
}
constexpr int pair_b(int p) { return p - pair_a(p) * (pair_a(p) - 1) / 2; }

template <int KMAX, int C, int L>
__device__ __forceinline__ void gram_fill(double (&vals)[64], const double (&q)[KMAX]) {
  if constexpr (L < 64) {
    constexpr int NP = (KMAX - 1) * (KMAX - 2) / 2;
    constexpr int p = C * 64 + L;
    if constexpr (p < NP)
      vals[L] = q[pair_a(p)] * q[pair_b(p)];
    else
      vals[L] = 0.0;
    gram_fill<KMAX, C, L + 1>(vals, q);
  }
}

// Add the products of every pair (a, b), b < a < KMAX-1, summed over the 64
// rows of this wave, to acc[pair]; 64 pairs per multi_reduce.
template <int KMAX, int C>
__device__ __forceinline__ void gram_chunks(const double (&q)[KMAX], double* acc) {
  constexpr int NP = (KMAX - 1) * (KMAX - 2) / 2;
  if constexpr (C * 64 < NP) {
    double vals[64];
    gram_fill<KMAX, C, 0>(vals, q);
    const double r = multi_reduce<64>(vals);
    const int lane = threadIdx.x & 63;
    if (C * 64 + lane < NP) acc[C * 64 + lane] += r;
    gram_chunks<KMAX, C + 1>(q, acc);
  }
}

// Per row: x <- q_0; for j < k-1: (q_j, x) <- (c x + s q_{j+1}, -s x + c q_{j+1}).
// The k values of the row are loaded first (registers), so the loads do not
// wait on the stores.  ICWY (gram): the k-1 rotated values also feed the
// strict lower Gram matrix, one pair-sum per (a, b), reduced with multi_reduce.
template <int KMAX, bool GRAM>
__global__ __launch_bounds__(kWG) void k_rotate(RotArgs a, Small sm, Tail t) {
  constexpr int NP = (KMAX - 1) * (KMAX - 2) / 2 > 0 ? (KMAX - 1) * (KMAX - 2) / 2 : 1;
  constexpr int NPA = GRAM ? NP : 1;
  __shared__ double s_c[KMAX], s_s[KMAX];
  __shared__ double s_acc[GRAM ? kWaves * NPA : 1];
  __shared__ double s_red[GRAM ? NPA : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cap = sm.cap;
  for (int j = threadIdx.x; j < KMAX; j += kWG) {
    s_c[j] = (j < a.k - 1) ? a.givens[j] : 1.0;
    s_s[j] = (j < a.k - 1) ? a.givens[cap + j] : 0.0;
  }
  if (GRAM)
    for (int c = threadIdx.x; c < kWaves * NPA; c += kWG) s_acc[c] = 0.0;
  __syncthreads();
  const int kk = a.k - 1;
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kWG + threadIdx.x;
    const bool valid = row < a.n;
    double q[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      q[j] = (j < a.k && valid) ? a.Q[(int64_t)j * a.ldq + row] : 0.0;
    double x = q[0];
#pragma unroll
    for (int j = 0; j < KMAX - 1; ++j) {
      if (j < kk) {
        const double y = q[j + 1];
        const double c = s_c[j], s = s_s[j];
        q[j] = c * x + s * y;
        x = -s * x + c * y;
      }
    }
    if (valid) {
#pragma unroll
      for (int j = 0; j < KMAX - 1; ++j)
        if (j < kk) a.Q[(int64_t)j * a.ldq + row] = q[j];
    }
    if (GRAM) {
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j >= kk) q[j] = 0.0;
      gram_chunks<KMAX, 0>(q, s_acc + w * NPA);
    }
  }
  if (GRAM) finish(sm, t, kk * (kk - 1) / 2, s_acc, NPA, s_red);
}

// ---------------------------------------------------------------------------
// elementwise passes
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWG) void k_scale(ScaleArgs a, int* status) {
  const double d = a.R[a.kk + (size_t)a.kk * a.cap];
  const int64_t stride = (int64_t)gridDim.x * kWG;
  for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < a.n; r += stride)
    a.out[r] = a.in[r] / d;
}

// i >= 1 (Alg. 1): f = g - x; Delta f = f - f_prev -> W; Delta g = g - g_prev
// -> ring slot; f_prev <- f; g_prev <- g; red[0] = ||f||^2.
// i == 0: f_prev = g - x, g_prev = g, x_next = g; red = [||f||^2, ||x_1-x_0||^2].
__global__ __launch_bounds__(kWG) void k_history(HistArgs a, Small sm, Tail t) {
  __shared__ double s_acc[kWaves * 2];
  __shared__ double s_red[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x < kWaves * 2) s_acc[threadIdx.x] = 0.0;
  __syncthreads();
  const int64_t ntiles = (a.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kTile + threadIdx.x;
    const bool full = (tile + 1) * kTile <= a.n;
    double xv[kRPT], gv[kRPT], f[kRPT];
    load_rows(xv, a.x, base, a.n, full);
    load_rows(gv, a.g, base, a.n, full);
#pragma unroll
    for (int i = 0; i < kRPT; ++i) f[i] = gv[i] - xv[i];
    if (a.first) {
      store_rows(f, a.f_prev, base, a.n, full);
      store_rows(gv, a.g_prev, base, a.n, full);
      store_rows(gv, a.x_next, base, a.n, full);
    } else {
      double fp[kRPT], gp[kRPT];
      load_rows(fp, a.f_prev, base, a.n, full);
      load_rows(gp, a.g_prev, base, a.n, full);
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        fp[i] = f[i] - fp[i];
        gp[i] = gv[i] - gp[i];
      }
      store_rows(fp, a.W, base, a.n, full);
      store_rows(gp, a.dg, base, a.n, full);
      store_rows(f, a.f_prev, base, a.n, full);
      store_rows(gv, a.g_prev, base, a.n, full);
    }
    const double p = wave_sum(dot_rows(f, f));
    if (lane == 0) {
      s_acc[w * 2] += p;
      s_acc[w * 2 + 1] += p;  // first step: x_1 - x_0 = f_0
    }
  }
  finish(sm, t, a.first ? 2 : 1, s_acc, 2, s_red);
}

// Alg. 1: x_{i+1} = g_i - sum_j gamma_j Delta g_{i-m_i+j}; red[0] = ||x_{i+1}-x_i||^2.
__global__ __launch_bounds__(kWG) void k_xupdate(XupdArgs a, Small sm, Tail t) {
  __shared__ double s_g[kMaxCols];
  __shared__ int s_slot[kMaxCols];
  __shared__ double s_acc[kWaves];
  __shared__ double s_red[1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < a.mi; j += kWG) {
    s_g[j] = a.gamma[j];
    s_slot[j] = (a.slot0 + j) % a.m;
  }
  if (threadIdx.x < kWaves) s_acc[threadIdx.x] = 0.0;
  __syncthreads();
  const int64_t ntiles = (a.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kTile + threadIdx.x;
    const bool full = (tile + 1) * kTile <= a.n;
    double gv[kRPT], xv[kRPT], acc[kRPT];
    load_rows(gv, a.g, base, a.n, full);
    load_rows(xv, a.x, base, a.n, full);
#pragma unroll
    for (int i = 0; i < kRPT; ++i) acc[i] = 0.0;
#pragma unroll 2
    for (int j = 0; j < a.mi; ++j) {
      double dv[kRPT];
      load_rows(dv, a.ring + (int64_t)s_slot[j] * a.ldq, base, a.n, full);
      const double gj = s_g[j];
#pragma unroll
      for (int i = 0; i < kRPT; ++i) acc[i] = fma(dv[i], gj, acc[i]);
    }
    double d2 = 0.0;
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const double xn = gv[i] - acc[i];
      const double d = xn - xv[i];
      d2 = fma(d, d, d2);
      gv[i] = xn;
    }
    store_rows(gv, a.x_next, base, a.n, full);
    const double p = wave_sum(d2);
    if (lane == 0) s_acc[w] += p;
  }
  finish(sm, t, 1, s_acc, 1, s_red);
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
    *sm.ticket = 0u;
  }
}

__global__ void k_copy(double* dst, const double* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int kmax_bucket(int k) { return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

hipError_t launch_dots(const DotsArgs& a, const Small& sm, const Tail& t, int grid,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return hipGetLastError();
}

hipError_t launch_update(const UpdArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return hipGetLastError();
}

hipError_t launch_cgs2b(const Cgs2bArgs& a, const Small& sm, const Tail& t, int grid,
                        hipStream_t st) {
  switch (kmax_bucket(a.k)) {
    case 8: hipLaunchKernelGGL(k_cgs2b<8>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    case 16: hipLaunchKernelGGL(k_cgs2b<16>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    case 32: hipLaunchKernelGGL(k_cgs2b<32>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    default: hipLaunchKernelGGL(k_cgs2b<64>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
  }
  return hipGetLastError();
}

hipError_t launch_givens(const Small& sm, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, sm, k);
  return hipGetLastError();
}

hipError_t launch_rotate(const RotArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  const int b = a.k <= 8 ? 8 : a.k <= 16 ? 16 : a.k <= 32 ? 32 : a.k <= 64 ? 64 : 65;
  if (a.gram) {
    switch (b) {
      case 8: hipLaunchKernelGGL((k_rotate<8, true>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 16: hipLaunchKernelGGL((k_rotate<16, true>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 32: hipLaunchKernelGGL((k_rotate<32, true>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 64: hipLaunchKernelGGL((k_rotate<64, true>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      default: return hipErrorInvalidValue;  // ICWY window limited to 64
    }
  } else {
    switch (b) {
      case 8: hipLaunchKernelGGL((k_rotate<8, false>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 16: hipLaunchKernelGGL((k_rotate<16, false>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 32: hipLaunchKernelGGL((k_rotate<32, false>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      case 64: hipLaunchKernelGGL((k_rotate<64, false>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
      default: hipLaunchKernelGGL((k_rotate<65, false>), dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_scale(const ScaleArgs& a, const Small& sm, hipStream_t st) {
  int64_t blocks = (a.n + kWG - 1) / kWG;
  int grid = (int)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_scale, dim3(grid), dim3(kWG), 0, st, a, sm.status);
  return hipGetLastError();
}

hipError_t launch_history(const HistArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_history, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return hipGetLastError();
}

hipError_t launch_xupdate(const XupdArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_xupdate, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return hipGetLastError();
}

hipError_t launch_init_small(const Small& sm, hipStream_t st) {
  hipLaunchKernelGGL(k_init_small, dim3(8), dim3(kWG), 0, st, sm);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  int64_t blocks = (n + kWG - 1) / kWG;
  int grid = (int)(blocks < 4096 ? blocks : 4096);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kWG), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace aa
