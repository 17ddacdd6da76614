// aa_kernels.hip -- FP64 HIP kernels for gfx950 of the windowed-QR Anderson
// acceleration update (Lockhart et al., arXiv 2110.09667, Algs. 1-6).
//
// Every kernel streams the tall-skinny n x k basis Q (column-major, padded
// leading dimension) from HBM once per pass.  A "Sync" of the paper -- a
// global reduction -- is one kernel: each workgroup folds its rows into
// per-wave partial sums in LDS, publishes one partial per reduced value, and
// a one-workgroup finalize kernel sums the partials in a fixed order and runs
// the small dense tail on the device (R and T updates, the T solve of ICWY,
// the back substitution for gamma).  Results are therefore bitwise
// reproducible for a given grid, and no value crosses to the host.
#include <math.h>

#include <type_traits>

#include "aa_device.h"

namespace aa {

// ---------------------------------------------------------------------------
// grid-wide reduction by the last-arriving workgroup, and the dense tails
// ---------------------------------------------------------------------------

__device__ void run_tail(const Small& sm, const Tail& t, const double* red) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int nthr = blockDim.x;
  const int cap = sm.cap;
  double* R = sm.R;
  double* T = sm.T;
  const int k = t.k;
  switch (t.op) {
    case TAIL_STORE:
      for (int i = tid; i < t.count; i += nthr) sm.coef0[i] = red[i];
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
      for (int i = tid; i < k; i += nthr) sm.coef0[i] = red[i];
      break;
    case TAIL_CGS2_Z:
      for (int i = tid; i < k; i += nthr) {
        sm.coef1[i] = red[i];
        R[i + (size_t)k * cap] = sm.coef0[i] + red[i];
      }
      break;
    case TAIL_ICWY:
      // Alg. 4: row k-1 of T is red[k + b] (b < k-1), diagonal 1; solve the
      // unit lower triangular T r' = r with r = red[0:k] (forward
      // substitution, one lane per row); r' is column k of R and the
      // coefficients of the update pass.
      for (int b = tid; b < k - 1; b += nthr) T[(k - 1) + (size_t)b * cap] = red[k + b];
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
      for (int i = tid; i < k; i += nthr) R[i + (size_t)k * cap] = red[i];
      if (t.reorth) {
        const int p = k - 1;
        const double scale = t.literal ? 1.0 : R[p + (size_t)p * cap];
        for (int i = tid; i < p; i += nthr) {
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
        for (int b = tid; b < a; b += nthr) T[a + (size_t)b * cap] = red[a * (a - 1) / 2 + b];
      break;
    }
    default:
      break;
  }
}

// Combine the per-wave accumulators of this workgroup and publish them as this
// workgroup's entries of the partials ([value][workgroup]); k_finalize, the
// next kernel on the stream, reduces them (the kernel boundary orders the
// writes before the reads, so no fence or atomic is needed here).
__device__ void finish(const Small& sm, int nred, const double* acc, int acc_stride) {
  __syncthreads();
  const int G = gridDim.x, b = blockIdx.x;
  for (int c = threadIdx.x; c < nred; c += kWG) {
    double s = acc[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += acc[w * acc_stride + c];
    sm.partials[(size_t)c * G + b] = s;
  }
}

// Fixed-order sum of the G partials of each of the nred values (one wave per
// value, lanes strided over the workgroups), then the dense tail.
__global__ __launch_bounds__(kFinWG) void k_finalize(Small sm, Tail t, int nred, int G) {
  __shared__ double red[kMaxRedAll];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int waves = kFinWG / 64;
  for (int c = w; c < nred; c += waves) {
    const double* p = sm.partials + (size_t)c * G;
    double s = 0.0;
    for (int g = lane; g < G; g += 64) s += p[g];
    s = wave_sum(s);
    if (lane == 0) red[c] = s;
  }
  __syncthreads();
  run_tail(sm, t, red);
}

// Visit the tiles of this workgroup: full tiles take the unmasked body.
template <class Body>
__device__ __forceinline__ void for_tiles(int64_t n, Body&& body) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t b2 = tile * kTile + 2 * (int64_t)threadIdx.x;
    if ((tile + 1) * kTile <= n)
      body(b2, std::true_type{});
    else
      body(b2, std::false_type{});
  }
}

// ---------------------------------------------------------------------------
// block dot products: red = [Q^T x, Q_{:,0:ny-1}^T y, x^T x]
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWG) void k_dots(DotsArgs a, Small sm, Tail t) {
  __shared__ double s_acc[kWaves * kMaxRed];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nq = a.nx > a.ny ? a.nx : a.ny;
  const int nred = a.nx + a.ny + (a.xx ? 1 : 0);
  for (int c = threadIdx.x; c < kWaves * kMaxRed; c += kWG) s_acc[c] = 0.0;
  __syncthreads();
  double* acc = s_acc + w * kMaxRed;
  for_tiles(a.n, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 xv[kPairs], yv[kPairs];
    ld2<F>(xv, a.x, b2, a.n);
    if (a.ny > 0) ld2<F>(yv, a.y, b2, a.n);
    if (a.xx) {
      const double p = wave_sum(dot2(xv, xv));
      if (lane == 0) acc[a.nx + a.ny] += p;
    }
    for (int j0 = 0; j0 < nq; j0 += kGroup) {
      double2 q[kGroup][kPairs];
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        if (j0 + c < nq)
          ld2<F>(q[c], a.Q + (int64_t)(j0 + c) * a.ldq, b2, a.n);
        else
          zero2(q[c]);
      }
      if (a.ny > 0) {
        double v[2 * kGroup];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
          v[c] = (j0 + c < a.nx) ? dot2(q[c], xv) : 0.0;
          v[kGroup + c] = (j0 + c < a.ny) ? dot2(q[c], yv) : 0.0;
        }
        const double r = multi_reduce<2 * kGroup>(v);
        if (lane < kGroup) {
          if (j0 + lane < a.nx) acc[j0 + lane] += r;
        } else if (lane < 2 * kGroup) {
          const int j = j0 + lane - kGroup;
          if (j < a.ny) acc[a.nx + j] += r;
        }
      } else {
        double v[kGroup];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) v[c] = (j0 + c < a.nx) ? dot2(q[c], xv) : 0.0;
        const double r = multi_reduce<kGroup>(v);
        if (lane < kGroup && j0 + lane < a.nx) acc[j0 + lane] += r;
      }
    }
  });
  finish(sm, nred, s_acc, kMaxRed);
}

// ---------------------------------------------------------------------------
// vector update out = v - Q c (+ fused dot / norm); DCGS-2 reorthogonalization
// ---------------------------------------------------------------------------

// acc1 += sum_{j in [j0, j1)} Q_j c1[j], acc2 += sum Q_j c2[j] (c2 may be null)
template <bool F>
__device__ __forceinline__ void combine_cols(const double* __restrict__ Q, int64_t ldq,
                                             int64_t b2, int64_t n, int j0, int j1,
                                             const double* c1, const double* c2,
                                             double2 (&acc1)[kPairs], double2 (&acc2)[kPairs]) {
  for (int g = j0; g < j1; g += kGroup) {
    double2 q[kGroup][kPairs];
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      if (g + c < j1)
        ld2<F>(q[c], Q + (int64_t)(g + c) * ldq, b2, n);
      else
        zero2(q[c]);
    }
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      if (g + c < j1) {
        axpy2(acc1, q[c], c1[g + c]);
        if (c2) axpy2(acc2, q[c], c2[g + c]);
      }
    }
  }
}

__global__ __launch_bounds__(kWG) void k_update(UpdArgs a, Small sm, Tail t) {
  __shared__ double s_c1[kMaxCols], s_c2[kMaxCols], s_s[kMaxCols];
  __shared__ double s_acc[kWaves * 4];
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
  const double* c2 = a.c2 ? s_c2 : nullptr;
  for_tiles(a.n, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 o[kPairs], dq[kPairs], acc1[kPairs], acc2[kPairs];
    ld2<F>(o, a.v, b2, a.n);
    if (a.dotcol >= 0) ld2<F>(dq, a.Q + (int64_t)a.dotcol * a.ldq, b2, a.n);
    zero2(acc1);
    zero2(acc2);
    if (a.dcgs2_p >= 0) {
      // Alg. 6: q'_p = q_p - Q_{:,0:p-1} s, then v - Q_{:,0:p-1} c - q'_p c_p
      const int p = a.dcgs2_p;
      double2 qp[kPairs];
      ld2<F>(qp, a.Q + (int64_t)p * a.ldq, b2, a.n);
      combine_cols<F>(a.Q, a.ldq, b2, a.n, 0, p, s_c1, a.reorth ? s_s : nullptr, acc1, acc2);
      if (a.reorth) {
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
          qp[i].x -= acc2[i].x;
          qp[i].y -= acc2[i].y;
        }
        st2<F>(qp, a.Qw + (int64_t)p * a.ldq, b2, a.n);
      }
      const double cp = s_c1[p];
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        o[i].x = (o[i].x - acc1[i].x) - qp[i].x * cp;
        o[i].y = (o[i].y - acc1[i].y) - qp[i].y * cp;
      }
    } else {
      combine_cols<F>(a.Q, a.ldq, b2, a.n, a.j0, a.j0 + a.nc, s_c1, c2, acc1, acc2);
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        o[i].x = (o[i].x - acc1[i].x) - acc2[i].x;
        o[i].y = (o[i].y - acc1[i].y) - acc2[i].y;
      }
    }
    if (a.out) st2<F>(o, a.out, b2, a.n);
    if (a.dotcol >= 0) {
      const double p = wave_sum(dot2(dq, o));
      if (lane == 0) s_acc[w * 4 + 0] += p;
    }
    if (a.nrm) {
      const double p = wave_sum(dot2(o, o));
      if (lane == 0) s_acc[w * 4 + inorm] += p;
    }
  });
  finish(sm, nred, s_acc, 4);
}

// ---------------------------------------------------------------------------
// CGS-2 second pass (Alg. 5): y = v - Q s in registers, red[j] = q_j^T y.
// One row per thread, the row's k values of Q held in registers.
// ---------------------------------------------------------------------------

template <int KMAX>
__global__ __launch_bounds__(kWG) void k_cgs2b(Cgs2bArgs a, Small sm, Tail t) {
  __shared__ double s_s[KMAX];
  __shared__ double s_acc[kWaves * KMAX];
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
  finish(sm, a.k, s_acc, KMAX);
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

// Per row: x <- q_0; for j < k-1: (q_j, x) <- (c x + s q_{j+1}, -s x + c q_{j+1}).
// The k values of the row are loaded first (registers), so the loads do not
// wait on the stores.
template <int KMAX>
__device__ __forceinline__ void rotate_row(double (&q)[KMAX], const RotArgs& a, int64_t row,
                                           bool valid, const double* s_c, const double* s_s) {
  const int kk = a.k - 1;
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
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    if (j >= kk) q[j] = 0.0;
}

template <int KMAX>
__global__ __launch_bounds__(kWG) void k_rotate(RotArgs a, Small sm, Tail t) {
  __shared__ double s_c[KMAX], s_s[KMAX];
  const int cap = sm.cap;
  for (int j = threadIdx.x; j < KMAX; j += kWG) {
    s_c[j] = (j < a.k - 1) ? a.givens[j] : 1.0;
    s_s[j] = (j < a.k - 1) ? a.givens[cap + j] : 0.0;
  }
  __syncthreads();
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kWG + threadIdx.x;
    double q[KMAX];
    rotate_row<KMAX>(q, a, row, row < a.n, s_c, s_s);
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// ICWY after QRDelete (Sec. 3.2): rotate, then accumulate the strict lower
// Gram matrix of the k-1 rotated columns, T_ab = q_a^T q_b (b < a).  The Gram
// over rows is a dense contraction, done on the matrix cores: each wave stages
// its 64 rotated rows in LDS (row stride KMAX + 1 doubles) and, 4 rows at a
// time, issues v_mfma_f64_16x16x4 on every lower pair of 16-column blocks.
// Operand layout of that instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; lane l, register r of the result holds D[l / 16 + 4 r]
// [l % 16].  Accumulators stay in registers across the workgroup's tiles; the
// workgroup reduces once at the end.
template <int KMAX>
__global__ __launch_bounds__(kWG) void k_rotate_gram(RotArgs a, Small sm, Tail t) {
  static_assert(KMAX % 16 == 0, "Gram blocks are 16 columns wide");
  constexpr int KP = KMAX + 1;
  constexpr int NB = KMAX / 16;
  constexpr int NBP = NB * (NB + 1) / 2;
  constexpr int NP = KMAX * (KMAX - 1) / 2;
  constexpr int STAGE = kWaves * 64 * KP;
  constexpr int ACC = kWaves * NP;
  __shared__ double s_buf[STAGE > ACC ? STAGE : ACC];
  __shared__ double s_c[KMAX], s_s[KMAX];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cap = sm.cap;
  for (int j = threadIdx.x; j < KMAX; j += kWG) {
    s_c[j] = (j < a.k - 1) ? a.givens[j] : 1.0;
    s_s[j] = (j < a.k - 1) ? a.givens[cap + j] : 0.0;
  }
  __syncthreads();
  v4d acc[NBP];
#pragma unroll
  for (int p = 0; p < NBP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  double* stage = s_buf + w * 64 * KP;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kWG + threadIdx.x;
    double q[KMAX];
    rotate_row<KMAX>(q, a, row, row < a.n, s_c, s_s);
#pragma unroll
    for (int j = 0; j < KMAX; ++j) stage[lane * KP + j] = q[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
    for (int r0 = 0; r0 < 64; r0 += 4) {
      double v[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) v[b] = stage[(r0 + lk) * KP + b * 16 + li];
      int p = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj <= bi; ++bj, ++p)
          acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[p], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();  // staging area becomes the per-wave pair accumulators
  double* accw = s_buf + w * NP;
  int p = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj <= bi; ++bj, ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ia = bi * 16 + lk + 4 * r, ib = bj * 16 + li;
        if (ia > ib) accw[ia * (ia - 1) / 2 + ib] = acc[p][r];
      }
  const int kk = a.k - 1;
  finish(sm, kk * (kk - 1) / 2, s_buf, NP);
}

// ---------------------------------------------------------------------------
// elementwise passes
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWG) void k_scale(ScaleArgs a, int* status) {
  const double d = a.R[a.kk + (size_t)a.kk * a.cap];
  const int64_t npair = a.n / 2;
  const int64_t stride = (int64_t)gridDim.x * kWG;
  const double2* in2 = reinterpret_cast<const double2*>(a.in);
  double2* out2 = reinterpret_cast<double2*>(a.out);
  for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < npair; r += stride) {
    const double2 v = in2[r];
    out2[r] = make_double2(v.x / d, v.y / d);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (a.n & 1)) a.out[a.n - 1] = a.in[a.n - 1] / d;
}

// i >= 1 (Alg. 1): f = g - x; Delta f = f - f_prev -> W; Delta g = g - g_prev
// -> ring slot; f_prev <- f; g_prev <- g; red[0] = ||f||^2.
// i == 0: f_prev = g - x, g_prev = g, x_next = g; red = [||f||^2, ||x_1-x_0||^2].
__global__ __launch_bounds__(kWG) void k_history(HistArgs a, Small sm, Tail t) {
  __shared__ double s_acc[kWaves * 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x < kWaves * 2) s_acc[threadIdx.x] = 0.0;
  __syncthreads();
  for_tiles(a.n, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 xv[kPairs], gv[kPairs], f[kPairs];
    ld2<F>(xv, a.x, b2, a.n);
    ld2<F>(gv, a.g, b2, a.n);
    if (a.first) {
#pragma unroll
      for (int i = 0; i < kPairs; ++i) f[i] = make_double2(gv[i].x - xv[i].x, gv[i].y - xv[i].y);
      st2<F>(f, a.f_prev, b2, a.n);
      st2<F>(gv, a.g_prev, b2, a.n);
      st2<F>(gv, a.x_next, b2, a.n);
    } else {
      double2 fp[kPairs], gp[kPairs];
      ld2<F>(fp, a.f_prev, b2, a.n);
      ld2<F>(gp, a.g_prev, b2, a.n);
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        f[i] = make_double2(gv[i].x - xv[i].x, gv[i].y - xv[i].y);
        fp[i] = make_double2(f[i].x - fp[i].x, f[i].y - fp[i].y);
        gp[i] = make_double2(gv[i].x - gp[i].x, gv[i].y - gp[i].y);
      }
      st2<F>(fp, a.W, b2, a.n);
      st2<F>(gp, a.dg, b2, a.n);
      st2<F>(f, a.f_prev, b2, a.n);
      st2<F>(gv, a.g_prev, b2, a.n);
    }
    const double p = wave_sum(dot2(f, f));
    if (lane == 0) {
      s_acc[w * 2] += p;
      s_acc[w * 2 + 1] += p;  // first step: x_1 - x_0 = f_0
    }
  });
  finish(sm, a.first ? 2 : 1, s_acc, 2);
}

// Alg. 1: x_{i+1} = g_i - sum_j gamma_j Delta g_{i-m_i+j}; red[0] = ||x_{i+1}-x_i||^2.
__global__ __launch_bounds__(kWG) void k_xupdate(XupdArgs a, Small sm, Tail t) {
  __shared__ double s_g[kMaxCols];
  __shared__ int s_slot[kMaxCols];
  __shared__ double s_acc[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < a.mi; j += kWG) {
    s_g[j] = a.gamma[j];
    s_slot[j] = (a.slot0 + j) % a.m;
  }
  if (threadIdx.x < kWaves) s_acc[threadIdx.x] = 0.0;
  __syncthreads();
  for_tiles(a.n, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 gv[kPairs], xv[kPairs], acc[kPairs];
    ld2<F>(gv, a.g, b2, a.n);
    ld2<F>(xv, a.x, b2, a.n);
    zero2(acc);
    for (int g0 = 0; g0 < a.mi; g0 += kGroup) {
      double2 d[kGroup][kPairs];
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        if (g0 + c < a.mi)
          ld2<F>(d[c], a.ring + (int64_t)s_slot[g0 + c] * a.ldq, b2, a.n);
        else
          zero2(d[c]);
      }
#pragma unroll
      for (int c = 0; c < kGroup; ++c)
        if (g0 + c < a.mi) axpy2(acc, d[c], s_g[g0 + c]);
    }
    double d2 = 0.0;
#pragma unroll
    for (int i = 0; i < kPairs; ++i) {
      const double2 xn = make_double2(gv[i].x - acc[i].x, gv[i].y - acc[i].y);
      const double dx = xn.x - xv[i].x, dy = xn.y - xv[i].y;
      d2 = fma(dx, dx, d2);
      d2 = fma(dy, dy, d2);
      gv[i] = xn;
    }
    st2<F>(gv, a.x_next, b2, a.n);
    const double p = wave_sum(d2);
    if (lane == 0) s_acc[w] += p;
  });
  finish(sm, 1, s_acc, 1);
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
  if (blockIdx.x == 0 && threadIdx.x == 0) *sm.status = AA_OK;
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

static hipError_t launch_finalize(const Small& sm, const Tail& t, int nred, int grid,
                                  hipStream_t st) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinWG), 0, st, sm, t, nred, grid);
  return hipGetLastError();
}

hipError_t launch_dots(const DotsArgs& a, const Small& sm, const Tail& t, int grid,
                       hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_dots, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return launch_finalize(sm, t, a.nx + a.ny + (a.xx ? 1 : 0), grid, st);
}

hipError_t launch_update(const UpdArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_update, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return launch_finalize(sm, t, (a.dotcol >= 0 ? 1 : 0) + (a.nrm ? 1 : 0), grid, st);
}

hipError_t launch_cgs2b(const Cgs2bArgs& a, const Small& sm, const Tail& t, int grid,
                        hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  switch (kmax_bucket(a.k)) {
    case 8: hipLaunchKernelGGL(k_cgs2b<8>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    case 16: hipLaunchKernelGGL(k_cgs2b<16>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    case 32: hipLaunchKernelGGL(k_cgs2b<32>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
    default: hipLaunchKernelGGL(k_cgs2b<64>, dim3(grid), dim3(kWG), 0, st, a, sm, t); break;
  }
  return launch_finalize(sm, t, a.k, grid, st);
}

hipError_t launch_givens(const Small& sm, int k, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, sm, k);
  return hipGetLastError();
}

hipError_t launch_rotate(const RotArgs& a, const Small& sm, const Tail& t, int grid,
                         hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  if (a.gram) {
    if (a.k <= 16)
      hipLaunchKernelGGL(k_rotate_gram<16>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else if (a.k <= 32)
      hipLaunchKernelGGL(k_rotate_gram<32>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else if (a.k <= 64)
      hipLaunchKernelGGL(k_rotate_gram<64>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else
      return hipErrorInvalidValue;  // the ICWY window is limited to 64 columns
    return launch_finalize(sm, t, (a.k - 1) * (a.k - 2) / 2, grid, st);
  } else {
    if (a.k <= 8)
      hipLaunchKernelGGL(k_rotate<8>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else if (a.k <= 16)
      hipLaunchKernelGGL(k_rotate<16>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else if (a.k <= 32)
      hipLaunchKernelGGL(k_rotate<32>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else if (a.k <= 64)
      hipLaunchKernelGGL(k_rotate<64>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
    else
      hipLaunchKernelGGL(k_rotate<65>, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  }
  return hipGetLastError();
}

hipError_t launch_scale(const ScaleArgs& a, const Small& sm, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (a.n + kWG - 1) / kWG;
  int grid = (int)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_scale, dim3(grid), dim3(kWG), 0, st, a, sm.status);
  return hipGetLastError();
}

hipError_t launch_history(const HistArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_history, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return launch_finalize(sm, t, a.first ? 2 : 1, grid, st);
}

hipError_t launch_xupdate(const XupdArgs& a, const Small& sm, const Tail& t, int grid,
                          hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_xupdate, dim3(grid), dim3(kWG), 0, st, a, sm, t);
  return launch_finalize(sm, t, 1, grid, st);
}

hipError_t launch_init_small(const Small& sm, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_init_small, dim3(8), dim3(kWG), 0, st, sm);
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
