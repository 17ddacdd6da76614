// aa_passes.h -- the passes of the windowed-QR AA update as tile-range bodies,
// shared by the grid-wide kernels (aa_kernels.hip: every workgroup takes tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... and publishes partial sums) and the
// workgroup-level step of the batched path (aa_batch.hip: one workgroup takes
// every tile of one instance and reduces in LDS).  Bodies accumulate into this
// wave's LDS accumulators; the caller zeroes them, combines the waves and runs
// the dense tail.  Block size is kWG (4 wave64s) throughout.
#pragma once

#include <type_traits>

#include "aa_device.h"

namespace aa {

// ---------------------------------------------------------------------------
// dense tails, run by one workgroup once the reduced values are in red[]
// ---------------------------------------------------------------------------

// Back substitution R gamma = c (Alg. 2, last line) by one wave: lane l < k1
// holds c_l in x on entry.  c is also kept in coef1 (free after QRAdd; the
// learned step reads it as a feature) unless keep_c is false (the lagged
// DCGS-2 solves before its update pass, which still reads coef1).  Threads
// past the first wave return.
__device__ __forceinline__ void rhs_backsolve(const Small& sm, int k1, double x,
                                              bool keep_c = true) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid >= 64) return;
  const int cap = sm.cap;
  if (keep_c && lane < k1) sm.coef1[lane] = x;
  double gam = 0.0;
  for (int a = k1 - 1; a >= 0; --a) {
    const double ga = __shfl(x, a, 64) / sm.R[a + (size_t)a * cap];
    if (lane < a) x -= sm.R[lane + (size_t)a * cap] * ga;
    if (lane == a) gam = ga;
  }
  if (lane < k1) sm.gamma[lane] = gam;
}

__device__ inline void run_tail(const Small& sm, const Tail& t, const double* red) {
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
    case TAIL_NORM: {
      const double nv = sqrt(red[t.idx]);
      if (tid == 0) {
        R[k + (size_t)k * cap] = nv;
        // breakdown: R_kk not above 64 eps times the column's norm (the
        // column numerically in the span of the window), or non-finite
        double col = nv * nv;
        for (int j = 0; j < k; ++j) col += R[j + (size_t)k * cap] * R[j + (size_t)k * cap];
        if (!(nv > kBreakdownRel * sqrt(col)) || !isfinite(nv)) *sm.status = AA_EBREAKDOWN;
      }
      if (t.rhs) {
        // c_k = q_k^T f = (w^T f) / R_kk; c_0..c_{k-1} were stashed in gamma
        // by the first pass of this QRAdd.  Then R gamma = c.
        __syncthreads();
        const double x = lane < k ? sm.gamma[lane] : (lane == k ? red[t.idx + 1] / nv : 0.0);
        __syncthreads();
        rhs_backsolve(sm, k + 1, x);
      }
      break;
    }
    case TAIL_CGS2_S:
      for (int i = tid; i < k; i += nthr) sm.coef0[i] = red[i];
      if (t.rhs)
        for (int i = tid; i < k; i += nthr) sm.gamma[i] = red[t.zoff + i];
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
      if (t.rhs)
        for (int i = tid; i < k; i += nthr) sm.gamma[i] = red[t.zoff + i];
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
      if (t.rhs) {
        // Q^T f with the columns as they stand after this add: only q_{k-1}
        // changes (q_{k-1} - Q_{:,0:k-2} s, not renormalized)
        for (int i = tid; i < k - 1; i += nthr) sm.gamma[i] = red[t.zoff + i];
        if (tid == 0) {
          double ck = red[t.zoff + k - 1];
          if (t.reorth)
            for (int i = 0; i < k - 1; ++i) ck -= red[k + i] * red[t.zoff + i];
          sm.gamma[k - 1] = ck;
        }
      }
      break;
    case TAIL_RHS:
      // Alg. 2, last line: back substitution R gamma = c, c = Q^T f_i
      rhs_backsolve(sm, k, lane < k ? red[lane] : 0.0);
      break;
    case TAIL_RES:
      if (tid == 0) {
        sm.scal[S_RES] = red[0];
        // the stopping test at the start of this iteration (reading A2):
        // the residual against ||f_0||, or the previous step's length
        if (sm.stop && sm.stop->done == 0) {
          const bool hit = t.stop_mode == kStopResidual
                               ? sqrt(red[0]) <= t.stop_tol * sqrt(sm.scal[S_RES0])
                               : (t.stop_mode == kStopStep && sqrt(sm.scal[S_STEP]) < t.stop_tol);
          if (hit) {
            sm.stop->iter = sm.stop->cur;
            sm.stop->k = t.k;
            sm.stop->m_i = t.m_i;
            sm.stop->done = AA_STOPPED_TEST;
          } else {
            sm.stop->cur += 1;  // iteration cur proceeds; the next one is cur + 1
          }
        }
      }
      break;
    case TAIL_FIRST:
      if (tid == 0) {
        sm.scal[S_RES] = red[0];
        sm.scal[S_RES0] = red[0];
        sm.scal[S_STEP] = red[1];
        if (sm.stop) sm.stop->cur = 1;  // the next iteration is i = 1
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
    case TAIL_DCGS2_LAG: {
      // DCGS-2 with the normalization lagged (Sec. 3.4), p = k-1 the newest
      // column.  red: Q^T v (z_j, j < p; beta at p), Q^T q_p (s_j; alpha at
      // k + p), v^T v at idx; with rhs Q^T f (c'_j; phi at zoff + p) and v^T f
      // at idx + 1.  One thread, in the order of the definition:
      //   rho = sqrt(alpha - s^T s); R_{0:p-1,p} += R_pp s; R_pp *= rho;
      //   R_{0:p-1,k} = z; R_pk = (beta - s^T z) / rho;
      //   R_kk = sqrt(nu - ||R_{0:p,k}||^2)   (no reduction over the new column).
      // The update pass then forms q_p = (q_p - Q s) / rho and
      // q_k = (v - Q z - q_p R_pk) / R_kk.
      const int p = k - 1;
      if (tid == 0) {
        double ss = 0.0, sz = 0.0;
        for (int j = 0; j < p; ++j) {
          const double sj = red[k + j];
          ss += sj * sj;
          sz += sj * red[j];
        }
        const double rho2 = red[k + p] - ss;
        const double rho = sqrt(rho2);
        const double rpp = R[p + (size_t)p * cap];
        for (int j = 0; j < p; ++j) R[j + (size_t)p * cap] += rpp * red[k + j];
        R[p + (size_t)p * cap] = rho * rpp;
        const double rpk = (red[p] - sz) / rho;
        double rr = 0.0;
        for (int j = 0; j < p; ++j) {
          const double zj = red[j];
          R[j + (size_t)k * cap] = zj;
          rr += zj * zj;
          sm.coef0[j] = zj;
          sm.coef1[j] = red[k + j];
        }
        R[p + (size_t)k * cap] = rpk;
        sm.coef0[p] = rpk;
        rr += rpk * rpk;
        const double w2 = red[t.idx] - rr;
        const double rkk = sqrt(w2);
        R[k + (size_t)k * cap] = rkk;
        sm.scal[S_RHO] = rho;
        sm.scal[S_RKK] = rkk;
        // the squared norms carry rounding of order eps times the squared
        // norm they are taken from: below 64 eps of it they are noise
        if (!(rho2 > kBreakdownRel * red[k + p]) || !isfinite(rho2) ||
            !(w2 > kBreakdownRel * red[t.idx]) || !isfinite(w2))
          *sm.status = AA_EBREAKDOWN;
        if (t.rhs) {
          // c = Q^T f of the grown basis from the same reduction: c_j = c'_j,
          // c_p = (phi - s^T c') / rho, c_k = (v^T f - z^T c' - R_pk c_p) / R_kk
          double sc = 0.0, zc = 0.0;
          for (int j = 0; j < p; ++j) {
            const double cj = red[t.zoff + j];
            sm.gamma[j] = cj;
            sc += red[k + j] * cj;
            zc += red[j] * cj;
          }
          const double cp = (red[t.zoff + p] - sc) / rho;
          sm.gamma[p] = cp;
          sm.gamma[k] = (red[t.idx + 1] - zc - rpk * cp) / rkk;
        }
      }
      if (t.rhs) {
        __syncthreads();
        const double x = lane <= k ? sm.gamma[lane] : 0.0;
        __syncthreads();
        rhs_backsolve(sm, k + 1, x, false);  // coef1 holds s for the update pass
      }
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// tile iteration
// ---------------------------------------------------------------------------

// Visit tiles t0, t0 + ts, ... of a streaming pass (kTile rows each); full
// tiles take the unmasked body.
template <class Body>
__device__ __forceinline__ void for_tiles(int64_t n, int64_t t0, int64_t ts, Body&& body) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t b2 = tile * kTile + 2 * (int64_t)threadIdx.x;
    if ((tile + 1) * kTile <= n)
      body(b2, std::true_type{});
    else
      body(b2, std::false_type{});
  }
}

// for_tiles, optionally from the last tile to the first (the same tiles per
// workgroup position, mirrored).
template <class Body>
__device__ __forceinline__ void for_tiles_dir(int64_t n, int64_t t0, int64_t ts, bool rev,
                                              Body&& body) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  for (int64_t it = t0; it < ntiles; it += ts) {
    const int64_t tile = rev ? ntiles - 1 - it : it;
    const int64_t b2 = tile * kTile + 2 * (int64_t)threadIdx.x;
    if ((tile + 1) * kTile <= n)
      body(b2, std::true_type{});
    else
      body(b2, std::false_type{});
  }
}

__device__ __forceinline__ void lds_zero(double* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// block dot products: acc_w[j] += Q_j^T x (j < nx); acc_w[nx + j] += Q_j^T y
// (j < ny); acc_w[nx + ny] += x^T x
// ---------------------------------------------------------------------------

__device__ __forceinline__ int dots_nred(const DotsArgs& a) {
  return a.nx + a.ny + a.nz + (a.xx ? 1 : 0) + (a.xz ? 1 : 0);
}

__device__ inline void dots_body(const DotsArgs& a, int64_t t0, int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  int nq = a.nx > a.ny ? a.nx : a.ny;
  if (a.nz > nq) nq = a.nz;
  double sxx = 0.0, sxz = 0.0;  // this lane's share of x^T x, x^T z
  for_tiles(a.n, t0, ts, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 xv[kPairs], yv[kPairs], zv[kPairs];
    ld2<F>(xv, a.x, b2, a.n);
    if (a.ny > 0) ld2<F>(yv, a.y, b2, a.n);
    if (a.nz > 0) ld2<F>(zv, a.z, b2, a.n);
    if (a.xx) sxx += dot2(xv, xv);
    if (a.xz) sxz += dot2(xv, zv);
    for (int j0 = 0; j0 < nq; j0 += kGroup) {
      double2 q[kGroup][kPairs];
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        if (j0 + c < nq)
          ld2<F>(q[c], a.Q + (int64_t)(j0 + c) * a.ldq, b2, a.n);
        else
          zero2(q[c]);
      }
      if (a.nz > 0) {
        // three right-hand sides: x, y, z (and a zero block to make 4 kGroup)
        double v[4 * kGroup];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
          v[c] = (j0 + c < a.nx) ? dot2(q[c], xv) : 0.0;
          v[kGroup + c] = (j0 + c < a.ny) ? dot2(q[c], yv) : 0.0;
          v[2 * kGroup + c] = (j0 + c < a.nz) ? dot2(q[c], zv) : 0.0;
          v[3 * kGroup + c] = 0.0;
        }
        const double r = multi_reduce<4 * kGroup>(v);
        if (lane < kGroup) {
          if (j0 + lane < a.nx) acc[j0 + lane] += r;
        } else if (lane < 2 * kGroup) {
          const int j = j0 + lane - kGroup;
          if (j < a.ny) acc[a.nx + j] += r;
        } else if (lane < 3 * kGroup) {
          const int j = j0 + lane - 2 * kGroup;
          if (j < a.nz) acc[a.nx + a.ny + j] += r;
        }
      } else if (a.ny > 0) {
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
  if (a.xx) {
    const double p = wave_sum(sxx);
    if (lane == 0) acc[a.nx + a.ny + a.nz] += p;
  }
  if (a.xz) {
    const double p = wave_sum(sxz);
    if (lane == 0) acc[a.nx + a.ny + a.nz + (a.xx ? 1 : 0)] += p;
  }
}

// Register-accumulated block dot products for at most KQ columns and NR
// right-hand sides (x; y when NR >= 2; z when NR == 3): each lane keeps its
// running sums of every (column, right-hand side) pair over all of its tiles,
// and each wave reduces them once at the end (one KQ-wide butterfly per
// right-hand side) instead of once per column group and tile.  Leaves the
// wave's sums in acc in dots_body's layout (x block, y block, z block, then
// x^T x).
template <int KQ, int NR>
__device__ inline void dots_reg_body(const DotsArgs& a, int64_t t0, int64_t ts, double* acc) {
  static_assert(KQ <= 64 && (KQ & (KQ - 1)) == 0 && NR >= 1 && NR <= 3, "bucket");
  const int lane = threadIdx.x & 63;
  int nq = a.nx > a.ny ? a.nx : a.ny;
  if (a.nz > nq) nq = a.nz;
  double s[NR][KQ];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < KQ; ++i) s[r][i] = 0.0;
  double sxx = 0.0, sxz = 0.0;
  // The QRAdd's first pass of ICWY and DCGS-2 dots Q with [v, q_{k-1}], and
  // q_{k-1} is Q's last column: take that column from the right-hand side
  // already in registers instead of reading it twice (the pass then moves
  // exactly its (k + 1) u; it read 4.6 % more).
  const int ylast = NR > 1 && a.ny > 0 && a.y == a.Q + (int64_t)(nq - 1) * a.ldq ? nq - 1 : -1;
  for_tiles(a.n, t0, ts, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 rv[NR][kPairs];
    // y (z) exists only when ny (nz) > 0: CGS-2 with the folded RHS has x and
    // z but no y, and its y pointer is null
    ld2<F>(rv[0], a.x, b2, a.n);
    if constexpr (NR > 1) {
      if (a.ny > 0) ld2<F>(rv[1], a.y, b2, a.n);
      else zero2(rv[1]);
    }
    if constexpr (NR > 2) {
      if (a.nz > 0) ld2<F>(rv[2], a.z, b2, a.n);
      else zero2(rv[2]);
    }
    if (a.xx) sxx += dot2(rv[0], rv[0]);
    if constexpr (NR > 2) {
      if (a.xz) sxz += dot2(rv[0], rv[2]);
    }
#pragma unroll
    for (int j0 = 0; j0 < KQ; j0 += kGroup) {
      if (j0 < nq) {
        double2 q[kGroup][kPairs];
#pragma unroll
        for (int c = 0; c < kGroup; ++c) {
          if (j0 + c == ylast) {
#pragma unroll
            for (int i = 0; i < kPairs; ++i) q[c][i] = rv[NR > 1 ? 1 : 0][i];
          } else if (j0 + c < nq) {
            ld2<F>(q[c], a.Q + (int64_t)(j0 + c) * a.ldq, b2, a.n);
          } else {
            zero2(q[c]);
          }
        }
#pragma unroll
        for (int c = 0; c < kGroup; ++c)
#pragma unroll
          for (int r = 0; r < NR; ++r) s[r][j0 + c] += dot2(q[c], rv[r]);
      }
    }
  });
  const int cnt[3] = {a.nx, a.ny, a.nz};
  int off = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double v = multi_reduce<KQ>(s[r]);  // lane l < KQ: column l over the wave
    if (lane < cnt[r]) acc[off + lane] = v;
    off += cnt[r];
  }
  if (a.xx) {
    const double p = wave_sum(sxx);
    if (lane == 0) acc[a.nx + a.ny + a.nz] = p;
  }
  if (a.xz) {
    const double p = wave_sum(sxz);
    if (lane == 0) acc[a.nx + a.ny + a.nz + (a.xx ? 1 : 0)] = p;
  }
}

// ---------------------------------------------------------------------------
// vector update out = v - Q c (+ fused dot / norm); DCGS-2 reorthogonalization
// acc_w[0] += Q_dotcol^T out (if dotcol >= 0); acc_w[inorm] += out^T out
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ int update_nred(const UpdArgs& a) {
  return (a.dotcol >= 0 ? 1 : 0) + (a.nrm ? 1 : 0) + (a.rhsv ? 1 : 0);
}

// Coefficients of an update pass copied to LDS (read once per workgroup).
__device__ inline void update_coefs(const UpdArgs& a, double* s_c1, double* s_c2, double* s_s) {
  for (int j = threadIdx.x; j < kMaxCols; j += blockDim.x) {
    s_c1[j] = (a.c1 && j < a.j0 + a.nc + 1) ? a.c1[j] : 0.0;
    s_c2[j] = (a.c2 && j < a.j0 + a.nc) ? a.c2[j] : 0.0;
    s_s[j] = (a.s && a.dcgs2_p >= 0 && j < a.dcgs2_p) ? a.s[j] : 0.0;
  }
}

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

__device__ inline void update_body(const UpdArgs& a, const double* s_c1, const double* s_c2,
                                   const double* s_s, int64_t t0, int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  const int inorm = a.dotcol >= 0 ? 1 : 0;
  const double* c2 = a.c2 ? s_c2 : nullptr;
  const double pdv = a.pdiv ? *a.pdiv : 1.0, odv = a.odiv ? *a.odiv : 1.0;
  double sdot = 0.0, snrm = 0.0, srhs = 0.0;  // this lane's running sums
  for_tiles_dir(a.n, t0, ts, a.rev != 0, [&](int64_t b2, auto full) {
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
        if (a.pdiv) {  // lagged DCGS-2: the normalization of q_p, one add late
#pragma unroll
          for (int i = 0; i < kPairs; ++i) {
            qp[i].x /= pdv;
            qp[i].y /= pdv;
          }
        }
        st2<F>(qp, a.Qw + (int64_t)p * a.ldq, b2, a.n);
      }
      const double cp = s_c1[p];
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        o[i].x = (o[i].x - acc1[i].x) - qp[i].x * cp;
        o[i].y = (o[i].y - acc1[i].y) - qp[i].y * cp;
      }
      if (a.odiv) {
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
          o[i].x /= odv;
          o[i].y /= odv;
        }
      }
    } else {
      combine_cols<F>(a.Q, a.ldq, b2, a.n, a.j0, a.j0 + a.nc, s_c1, c2, acc1, acc2);
#pragma unroll
      for (int i = 0; i < kPairs; ++i) {
        o[i].x = (o[i].x - acc1[i].x) - acc2[i].x;
        o[i].y = (o[i].y - acc1[i].y) - acc2[i].y;
      }
    }
    if (a.out) st2<F, AA_NT_STORE_UPDATE != 0>(o, a.out, b2, a.n);
    if (a.dotcol >= 0) sdot += dot2(dq, o);
    if (a.nrm) snrm += dot2(o, o);
    if (a.rhsv) {
      double2 fv[kPairs];
      ld2<F>(fv, a.rhsv, b2, a.n);
      srhs += dot2(fv, o);
    }
  });
  // one wave reduction per value, after all of this lane's tiles
  if (a.dotcol >= 0) {
    const double p = wave_sum(sdot);
    if (lane == 0) acc[0] += p;
  }
  if (a.nrm) {
    const double p = wave_sum(snrm);
    if (lane == 0) acc[inorm] += p;
  }
  if (a.rhsv) {
    const double p = wave_sum(srhs);
    if (lane == 0) acc[inorm + (a.nrm ? 1 : 0)] += p;
  }
}

// ---------------------------------------------------------------------------
// CGS-2 second pass (Alg. 5): y = v - Q s in registers, acc_w[j] += q_j^T y.
// One row per thread (tiles of kWG rows), the row's k values held in registers.
// ---------------------------------------------------------------------------

template <int KMAX>
__device__ inline void cgs2b_body(const Cgs2bArgs& a, const double* s_s, int64_t t0, int64_t ts,
                                  double* acc) {
  const int lane = threadIdx.x & 63;
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t it = t0; it < ntiles; it += ts) {
    const int64_t tile = a.rev ? ntiles - 1 - it : it;
    const int64_t row = tile * kWG + threadIdx.x;
    const bool valid = row < a.n;
    double q[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      q[j] = (j < a.k && valid) ? a.Q[(int64_t)j * a.ldq + row] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) s = fma(q[j], s_s[j], s);
    const double y = (valid ? a.v[row] : 0.0) - s;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) q[j] *= y;
    const double r = multi_reduce<KMAX>(q);
    if (lane < KMAX) acc[lane] += r;
  }
}

// The grid pass for at most KMAX columns on 16-byte row pairs (NP per lane
// per tile) with per-lane running sums and one KMAX-wide butterfly per wave
// at the end.  The one-row form above reduces every 256-row tile, which
// leaves too little in flight when k is small (k = 1 streamed 1.9 TB/s).
// The 32-column bucket takes one pair per lane (its 32 column pairs already
// keep 512 bytes per lane in flight, and two would not fit the registers).
template <bool FULL, int NP>
__device__ __forceinline__ void ld2n(double2 (&r)[NP], const double* __restrict__ p, int64_t b2,
                                     int64_t n) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int64_t row = b2 + (int64_t)i * 2 * kWG;
    if (FULL) {
      const f64x2 v = ld2v(reinterpret_cast<const double2*>(p + row));
      r[i] = make_double2(v.x, v.y);
    } else {
      r[i].x = row < n ? p[row] : 0.0;
      r[i].y = row + 1 < n ? p[row + 1] : 0.0;
    }
  }
}

template <int KMAX, int NP>
__device__ inline void cgs2b_pair_body(const Cgs2bArgs& a, const double* s_s, int64_t t0,
                                       int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  constexpr int64_t kRows = (int64_t)kWG * 2 * NP;  // rows per tile
  double sum[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) sum[j] = 0.0;
  auto body = [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 q[KMAX][NP];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < a.k) {
        ld2n<F, NP>(q[j], a.Q + (int64_t)j * a.ldq, b2, a.n);
      } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) q[j][i] = make_double2(0.0, 0.0);
      }
    }
    double2 y[NP];
    ld2n<F, NP>(y, a.v, b2, a.n);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        sx = fma(q[j][i].x, s_s[j], sx);
        sy = fma(q[j][i].y, s_s[j], sy);
      }
      y[i].x -= sx;
      y[i].y -= sy;
    }
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        d = fma(q[j][i].x, y[i].x, d);
        d = fma(q[j][i].y, y[i].y, d);
      }
      sum[j] += d;
    }
  };
  const int64_t ntiles = (a.n + kRows - 1) / kRows;
  for (int64_t it = t0; it < ntiles; it += ts) {
    const int64_t tile = a.rev ? ntiles - 1 - it : it;
    const int64_t b2 = tile * kRows + 2 * (int64_t)threadIdx.x;
    if ((tile + 1) * kRows <= a.n)
      body(b2, std::true_type{});
    else
      body(b2, std::false_type{});
  }
  const double r = multi_reduce<KMAX>(sum);
  if (lane < KMAX && lane < a.k) acc[lane] += r;
}

// The same pass with per-lane running sums (workgroup-level step, at most
// KMAX columns): per row the same y = v - Q s, then sum_j += q_j y over all of
// the lane's rows, and one KMAX-wide butterfly per wave at the end instead of
// one per tile.
template <int KMAX>
__device__ inline void cgs2b_reg_body(const Cgs2bArgs& a, const double* s_s, int64_t t0,
                                      int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  double sum[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) sum[j] = 0.0;
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t row = tile * kWG + threadIdx.x;
    const bool valid = row < a.n;
    double q[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      q[j] = (j < a.k && valid) ? a.Q[(int64_t)j * a.ldq + row] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) s = fma(q[j], s_s[j], s);
    const double y = (valid ? a.v[row] : 0.0) - s;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) sum[j] = fma(q[j], y, sum[j]);
  }
  const double r = multi_reduce<KMAX>(sum);
  if (lane < KMAX && lane < a.k) acc[lane] += r;
}

// The same pass without a k-wide register array (workgroup-level step): per
// 256-row tile, one sweep forms y = v - Q s, a second sweep over the same tile
// (cache-resident, just read) forms Q^T y in groups of kGroup columns.
__device__ inline void cgs2b_stream_body(const Cgs2bArgs& a, const double* s_s, int64_t t0,
                                         int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  const int64_t ntiles = (a.n + kWG - 1) / kWG;
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t row = tile * kWG + threadIdx.x;
    const bool valid = row < a.n;
    const double* qrow = a.Q + row;
    double s = 0.0;
    for (int j = 0; j < a.k; ++j) s = fma(valid ? qrow[(int64_t)j * a.ldq] : 0.0, s_s[j], s);
    const double y = (valid ? a.v[row] : 0.0) - s;
    for (int j0 = 0; j0 < a.k; j0 += kGroup) {
      double v[kGroup];
#pragma unroll
      for (int c = 0; c < kGroup; ++c)
        v[c] = (valid && j0 + c < a.k) ? qrow[(int64_t)(j0 + c) * a.ldq] * y : 0.0;
      const double r = multi_reduce<kGroup>(v);
      if (lane < kGroup && j0 + lane < a.k) acc[j0 + lane] += r;
    }
  }
}

// ---------------------------------------------------------------------------
// QRDelete (Alg. 2): Givens rotations from R, then one sweep over Q
// ---------------------------------------------------------------------------

// H = R_{:,1:k-1}; rotation j zeroes H_{j+1,j}; R <- the (k-1)x(k-1) triangle.
// Any block size; every thread must call (barriers inside).  H: k*k doubles
// of LDS.
__device__ inline void givens_body(const Small& sm, int k, double* H) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int cap = sm.cap;
  const int nc = k - 1;
  for (int idx = tid; idx < k * nc; idx += nthr) {
    const int i = idx % k, j = idx / k;
    H[i + j * k] = sm.R[i + (size_t)(j + 1) * cap];
  }
  __syncthreads();
  for (int j = 0; j < nc; ++j) {
    const double x = H[j + j * k], y = H[(j + 1) + j * k];
    const double rho = hypot(x, y);
    const double c = rho > 0.0 ? x / rho : 1.0;
    const double s = rho > 0.0 ? y / rho : 0.0;
    __syncthreads();
    for (int col = j + tid; col < nc; col += nthr) {
      const double hj = H[j + col * k], hj1 = H[(j + 1) + col * k];
      H[j + col * k] = c * hj + s * hj1;
      H[(j + 1) + col * k] = -s * hj + c * hj1;
    }
    if (tid == 0) {
      sm.givens[j] = c;
      sm.givens[cap + j] = s;
    }
    __syncthreads();
    if (tid == 0) H[(j + 1) + j * k] = 0.0;
    __syncthreads();
  }
  for (int idx = tid; idx < k * k; idx += nthr) {
    const int i = idx % k, j = idx / k;
    sm.R[i + (size_t)j * cap] = (i < nc && j < nc && i <= j) ? H[i + j * k] : 0.0;
  }
}

// ICWY's T after QRDelete without a reduction (AA_ICWY_T_TRANSFORM): the old
// Gram matrix S = I + L + L^T of columns 0..k-2 (L the strict lower part of T,
// whose rows 0..k-2 are current) is rotated like the columns of Q,
// S <- W^T S W by rotations 0..k-3 (column pair j, j+1, then row pair j, j+1);
// its strict lower rows 0..k-3 are the new T's (the new columns 0..k-3 mix old
// columns 0..k-2 only).  The last row belongs to the column old column k-1
// entered; the next QRAdd's first reduction recomputes it before any read
// (Alg. 4), so it is left alone.  After givens_body (coefficients in
// sm.givens); S: (k-1)^2 doubles of LDS; every thread must call.
__device__ inline void t_transform_body(const Small& sm, int k, double* S) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int cap = sm.cap, kk = k - 1;
  if (kk < 3) return;  // rows 0..kk-2 of a strict lower part: nothing below row 0
  for (int idx = tid; idx < kk * kk; idx += nthr) {
    const int a = idx % kk, b = idx / kk;
    S[idx] = a == b ? 1.0 : (a > b ? sm.T[a + (size_t)b * cap] : sm.T[b + (size_t)a * cap]);
  }
  __syncthreads();
  for (int j = 0; j + 1 < kk; ++j) {
    const double c = sm.givens[j], s = sm.givens[cap + j];
    for (int r = tid; r < kk; r += nthr) {
      const double x = S[r + j * kk], y = S[r + (j + 1) * kk];
      S[r + j * kk] = c * x + s * y;
      S[r + (j + 1) * kk] = -s * x + c * y;
    }
    __syncthreads();
    for (int r = tid; r < kk; r += nthr) {
      const double x = S[j + r * kk], y = S[(j + 1) + r * kk];
      S[j + r * kk] = c * x + s * y;
      S[(j + 1) + r * kk] = -s * x + c * y;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kk * kk; idx += nthr) {
    const int a = idx % kk, b = idx / kk;
    if (b < a && a < kk - 1) sm.T[a + (size_t)b * cap] = S[idx];
  }
}

__device__ inline void givens_coefs(const RotArgs& a, int cap, double* s_c, double* s_s, int kmax) {
  for (int j = threadIdx.x; j < kmax; j += blockDim.x) {
    s_c[j] = (j < a.k - 1) ? a.givens[j] : 1.0;
    s_s[j] = (j < a.k - 1) ? a.givens[cap + j] : 0.0;
  }
}

// Per row: x <- q_0; for j < k-1: (q_j, x) <- (c_j x + s_j q_{j+1},
// -s_j x + c_j q_{j+1}) -- rotation j of QRDelete applied to columns j, j+1
// of Q, in the order the rotations were generated.  The sweep streams the
// columns in chunks of CH with the next chunk's loads issued before the
// current chunk's stores (registers hold two chunks, not the whole row).
// Each rotated value is also passed to emit(j, value) (the ICWY Gram stages it).
// CH is the number of loads a lane keeps in flight: kernels that run few waves
// per SIMD (wide Gram staging) need a deeper chunk to keep HBM busy.
constexpr int kRotCh = 8;
// Load depth of the paired-row sweep of the plain rotation pass.
#ifndef AA_ROT_CH_PAIR
#define AA_ROT_CH_PAIR 8
#endif
constexpr int kRotChPair = AA_ROT_CH_PAIR;

// The first loads of a row's sweep (q_0 and the next CH columns), split off
// so that a caller can issue them early (rotate_gram_body fetches the next
// tile's while the matrix cores work on the current one).
template <int CH>
struct RotHead {
  double x;
  double nxt[CH];
};

template <int CH>
__device__ __forceinline__ void rot_head(const RotArgs& a, int64_t row, bool valid,
                                         RotHead<CH>& h) {
  const double* qrow = a.Q + row;
  h.x = valid ? ld1(qrow) : 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c)
    h.nxt[c] = (valid && 1 + c < a.k) ? ld1(qrow + (int64_t)(1 + c) * a.ldq) : 0.0;
}

template <int CH, class Emit>
__device__ __forceinline__ void rotate_row_from(const RotArgs& a, int64_t row, bool valid,
                                                const double* s_c, const double* s_s,
                                                RotHead<CH>& h, Emit&& emit) {
  const int kk = a.k - 1;
  const double* qrow = a.Q + row;
  double* qw = a.Q + row;
  double x = h.x;
  for (int j0 = 0; j0 < kk; j0 += CH) {
    double cur[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) cur[c] = h.nxt[c];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int jn = j0 + CH + 1 + c;
      h.nxt[c] = (valid && jn < a.k) ? ld1(qrow + (int64_t)jn * a.ldq) : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = j0 + c;
      if (j < kk) {
        const double y = cur[c];
        const double cj = s_c[j], sj = s_s[j];
        const double qn = cj * x + sj * y;
        x = -sj * x + cj * y;
        if (valid) st1_stream(qn, qw + (int64_t)j * a.ldq);
        emit(j, valid ? qn : 0.0);
      }
    }
  }
}

template <int CH = kRotCh, class Emit>
__device__ __forceinline__ void rotate_row(const RotArgs& a, int64_t row, bool valid,
                                           const double* s_c, const double* s_s, Emit&& emit) {
  RotHead<CH> h;
  rot_head<CH>(a, row, valid, h);
  rotate_row_from<CH>(a, row, valid, s_c, s_s, h, emit);
}

// The same sweep for two adjacent rows (row even, row + 1 < n) with 16-byte
// loads and stores.
template <int CH = kRotCh>
__device__ __forceinline__ void rotate_pair(const RotArgs& a, int64_t row, const double* s_c,
                                            const double* s_s) {
  const int kk = a.k - 1;
  const double* qrow = a.Q + row;
  f64x2 x = ld2v(reinterpret_cast<const double2*>(qrow));
  f64x2 nxt[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
    nxt[c] = (1 + c < a.k) ? ld2v(reinterpret_cast<const double2*>(qrow + (int64_t)(1 + c) * a.ldq))
                           : f64x2{0.0, 0.0};
  for (int j0 = 0; j0 < kk; j0 += CH) {
    f64x2 cur[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) cur[c] = nxt[c];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int jn = j0 + CH + 1 + c;
      nxt[c] = jn < a.k ? ld2v(reinterpret_cast<const double2*>(qrow + (int64_t)jn * a.ldq))
                        : f64x2{0.0, 0.0};
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = j0 + c;
      if (j < kk) {
        const f64x2 y = cur[c];
        const double cj = s_c[j], sj = s_s[j];
        f64x2 qn;
        qn.x = cj * x.x + sj * y.x;
        qn.y = cj * x.y + sj * y.y;
        x.x = -sj * x.x + cj * y.x;
        x.y = -sj * x.y + cj * y.y;
        st2v_stream(qn, a.Q + row + (int64_t)j * a.ldq);
      }
    }
  }
}

// Row pairs p = tile kWG + tid (rows 2p, 2p + 1); an odd last row alone.
// CH: load depth of the paired sweep.
template <int CH = kRotChPair>
__device__ inline void rotate_body(const RotArgs& a, const double* s_c, const double* s_s,
                                   int64_t t0, int64_t ts) {
  const int64_t npair = (a.n + 1) / 2;
  const int64_t ntiles = (npair + kWG - 1) / kWG;
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t row = 2 * (tile * kWG + threadIdx.x);
    if (row + 1 < a.n)
      rotate_pair<CH>(a, row, s_c, s_s);
    else if (row < a.n)
      rotate_row(a, row, true, s_c, s_s, [](int, double) {});
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KMAX>
struct GramShape {
  static_assert(KMAX % 16 == 0, "Gram blocks are 16 columns wide");
  static constexpr int KP = KMAX + 1;            // largest LDS row stride (doubles)
  static constexpr int NB = KMAX / 16;           // 16-column blocks
  static constexpr int NBP = NB * (NB + 1) / 2;  // lower block pairs
  static constexpr int NP = KMAX * (KMAX - 1) / 2;
  static constexpr int STAGE = kWaves * 64 * KP; // staging doubles per workgroup (largest)
};

// LDS row stride for kk staged columns: the smallest odd number >= kk, so
// that the 64 lanes of a wave writing one row each spread over all banks.
__host__ __device__ constexpr int gram_stride(int kk) { return kk | 1; }

// Staging doubles a workgroup of `waves` waves needs for kk staged columns
// (the same area later holds the per-wave pair sums).
__host__ __device__ constexpr int gram_lds_doubles(int kk, int waves = kWaves) {
  return waves * 64 * gram_stride(kk) > waves * (kk * (kk - 1) / 2)
             ? waves * 64 * gram_stride(kk)
             : waves * (kk * (kk - 1) / 2);
}

// ICWY after QRDelete (Sec. 3.2): rotate, then accumulate the strict lower
// Gram matrix of the kk = k-1 rotated columns, T_ab = q_a^T q_b (b < a)
// (with a.naug > 0 the staged rows also carry v and f after the kk columns,
// so the pairs (kk, b) and (kk + 1, b) are q_b^T v and q_b^T f).  The
// Gram over rows is a dense contraction, done on the matrix cores: each wave
// stages its 64 rotated rows in LDS (row stride kp = gram_stride(kk) doubles,
// only the kk live columns) and, 4 rows at a time, issues v_mfma_f64_16x16x4
// on every lower pair of 16-column blocks, reading zeros for the columns past
// kk.  Operand layout of that instruction: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; lane l, register r of the result holds
// D[l / 16 + 4 r][l % 16].  Accumulators stay in registers across all tiles.
// In the 64-column instance, block pairs whose row block lies wholly past the
// live columns are skipped (their accumulators stay zero; the narrower
// instances always have every block live).  CH is the rotation's load depth.
template <int KMAX, int WG = kWG, int CH = kRotCh>
__device__ inline void rotate_gram_body(const RotArgs& a, const double* s_c, const double* s_s,
                                        int64_t t0, int64_t ts, double* stage_all, int kp,
                                        v4d (&acc)[GramShape<KMAX>::NBP]) {
  using S = GramShape<KMAX>;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* stage = stage_all + w * 64 * kp;
#pragma unroll
  for (int p = 0; p < S::NBP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t ntiles = (a.n + WG - 1) / WG;
  const int kk = a.k - 1, na = gram_cols(a);
  bool live[S::NB];
#pragma unroll
  for (int b = 0; b < S::NB; ++b) live[b] = b * 16 + li < na;
  const int nbl = (na + 15) / 16;  // blocks holding a live column
  // PREFETCH (the 64-column instance, whose MFMA phase is long): the next
  // tile's first column loads are issued before this tile's MFMA phase
  // (m = 50 step 8.53 -> 8.36 ms; the narrower instances measured ~1.5 %
  // slower with it and keep the plain order).
  constexpr bool PREFETCH = KMAX >= 64;
  RotHead<CH> h;
  if (PREFETCH && t0 < ntiles) {
    const int64_t row = t0 * WG + threadIdx.x;
    rot_head<CH>(a, row, row < a.n, h);
  }
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t row = tile * WG + threadIdx.x;
    const bool valid = row < a.n;
    double* srow = stage + lane * kp;
    if (a.naug > 0) srow[kk] = valid ? ld1(a.v + row) : 0.0;
    if (a.naug > 1) srow[kk + 1] = valid ? ld1(a.f + row) : 0.0;
    if (!PREFETCH) rot_head<CH>(a, row, valid, h);
    rotate_row_from<CH>(a, row, valid, s_c, s_s, h, [&](int j, double v) {
      if (j < na) srow[j] = v;
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the next tile's first column loads, in flight during the MFMA phase
    if (PREFETCH && tile + ts < ntiles) {
      const int64_t nrow = (tile + ts) * WG + threadIdx.x;
      rot_head<CH>(a, nrow, nrow < a.n, h);
    }
#pragma unroll 4
    for (int r0 = 0; r0 < 64; r0 += 4) {
      double v[S::NB];
#pragma unroll
      for (int b = 0; b < S::NB; ++b) v[b] = live[b] ? stage[(r0 + lk) * kp + b * 16 + li] : 0.0;
      int p = 0;
#pragma unroll
      for (int bi = 0; bi < S::NB; ++bi)
#pragma unroll
        for (int bj = 0; bj <= bi; ++bj, ++p)
          if (KMAX < 64 || bi < nbl)
            acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[p], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Small windows (at most NAMAX staged columns): the same rotation and strict
// lower Gram without matrix cores.  Each lane takes a pair of rows (16-byte
// loads; an odd last row alone), loads its k columns at once, rotates them in
// registers and accumulates the pair products of the staged values z (the kk
// rotated columns, then v and f when a.naug > 0) in acc[i (i - 1) / 2 + j],
// j < i < na.  A 16 x 16 x 4 MFMA block spends 256 multiply-adds per row
// whatever the live columns; here a row costs na (na - 1) / 2, and FP64 MFMA
// runs no faster than the vector units.
template <int NAMAX, int NR, bool PAIR>
__device__ __forceinline__ void gram_small_rows(const RotArgs& a, const double* s_c,
                                                const double* s_s, int64_t row,
                                                double (&acc)[NR]) {
  const int kk = a.k - 1, na = gram_cols(a);
  auto load = [&](const double* p) -> f64x2 {
    if constexpr (PAIR) return ld2v(reinterpret_cast<const double2*>(p));
    else return f64x2{ld1(p), 0.0};
  };
  auto load_aug = [&](const double* p) -> f64x2 {
    if constexpr (PAIR) return f64x2{ld1(p), ld1(p + 1)};  // v, f: no alignment assumed
    else return f64x2{ld1(p), 0.0};
  };
  f64x2 q[NAMAX + 1];
#pragma unroll
  for (int j = 0; j <= NAMAX; ++j)
    q[j] = j <= kk ? load(a.Q + row + (int64_t)j * a.ldq) : f64x2{0.0, 0.0};
  const f64x2 v0 = a.naug > 0 ? load_aug(a.v + row) : f64x2{0.0, 0.0};
  const f64x2 v1 = a.naug > 1 ? load_aug(a.f + row) : f64x2{0.0, 0.0};
  f64x2 z[NAMAX];
  f64x2 x = q[0];
#pragma unroll
  for (int j = 0; j < NAMAX; ++j) {
    if (j < kk) {
      const f64x2 y = q[j + 1];
      const double cj = s_c[j], sj = s_s[j];
      f64x2 qn;
      qn.x = cj * x.x + sj * y.x;
      qn.y = cj * x.y + sj * y.y;
      x.x = -sj * x.x + cj * y.x;
      x.y = -sj * x.y + cj * y.y;
      double* qw = a.Q + row + (int64_t)j * a.ldq;
      if constexpr (PAIR) st2v_stream(qn, qw);
      else st1_stream(qn.x, qw);
      z[j] = qn;
    } else {
      z[j] = j == kk ? v0 : (j == kk + 1 ? v1 : f64x2{0.0, 0.0});
    }
  }
  int p = 0;
#pragma unroll
  for (int i = 1; i < NAMAX; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j, ++p)
      if (i < na) acc[p] += z[i].x * z[j].x + z[i].y * z[j].y;
}

template <int NAMAX, int NR>
__device__ inline void rotate_gram_small_body(const RotArgs& a, const double* s_c,
                                              const double* s_s, int64_t t0, int64_t ts,
                                              double (&acc)[NR]) {
  static_assert(NAMAX * (NAMAX - 1) / 2 <= NR, "pair accumulators");
#pragma unroll
  for (int p = 0; p < NR; ++p) acc[p] = 0.0;
  const int64_t npair = a.n / 2;
  for (int64_t pr = t0 * kWG + threadIdx.x; pr < npair; pr += ts * kWG)
    gram_small_rows<NAMAX, NR, true>(a, s_c, s_s, 2 * pr, acc);
  if ((a.n & 1) && t0 == 0 && threadIdx.x == 0)
    gram_small_rows<NAMAX, NR, false>(a, s_c, s_s, a.n - 1, acc);
}

// 33 to 64 staged columns with half the staging.  The rotation sweep of a row
// is resumed in two halves (rotations 0..31, then 32..kk-1), each half staged
// in a 64-row x 32-column LDS tile (row stride kHalfStride).  After the first
// half each lane keeps its MFMA operands of blocks 0 and 1 for all 16 row
// quads of the tile in registers (32 doubles), so the second half can pair
// blocks 2 and 3 with them.  Half the LDS of rotate_gram_body<64> per wave:
// twice the waves per compute unit.  Same pairs and accumulator order
// (p = bi (bi + 1) / 2 + bj), so gram_store<64> applies.
constexpr int kHalfStride = 33;

template <int WG, int CH>
__device__ inline void rotate_gram_split_body(const RotArgs& a, const double* s_c,
                                              const double* s_s, int64_t t0, int64_t ts,
                                              double* stage_all, v4d (&acc)[10]) {
  static_assert(32 % CH == 0, "the halves are whole chunks");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* stage = stage_all + w * 64 * kHalfStride;
  double* srow = stage + lane * kHalfStride;
#pragma unroll
  for (int p = 0; p < 10; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t ntiles = (a.n + WG - 1) / WG;
  const int kk = a.k - 1, na = gram_cols(a);  // 32 < na <= 64
  const bool live2 = 32 + li < na, live3 = 48 + li < na, blk3 = na > 48;
  for (int64_t tile = t0; tile < ntiles; tile += ts) {
    const int64_t row = tile * WG + threadIdx.x;
    const bool valid = row < a.n;
    const double* qrow = a.Q + row;
    double* qw = a.Q + row;
    const double av = (valid && a.naug > 0) ? ld1(a.v + row) : 0.0;
    const double af = (valid && a.naug > 1) ? ld1(a.f + row) : 0.0;
    double x = valid ? ld1(qrow) : 0.0;
    double nxt[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c)
      nxt[c] = (valid && 1 + c < a.k) ? ld1(qrow + (int64_t)(1 + c) * a.ldq) : 0.0;
    // rotations jb .. min(je, kk) - 1, rotated column j staged at j - base
    auto sweep = [&](int jb, int je, int base) {
      for (int j0 = jb; j0 < je && j0 < kk; j0 += CH) {
        double cur[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) cur[c] = nxt[c];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int jn = j0 + CH + 1 + c;
          nxt[c] = (valid && jn < a.k) ? ld1(qrow + (int64_t)jn * a.ldq) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int j = j0 + c;
          if (j < kk) {
            const double y = cur[c];
            const double cj = s_c[j], sj = s_s[j];
            const double qn = cj * x + sj * y;
            x = -sj * x + cj * y;
            if (valid) st1_stream(qn, qw + (int64_t)j * a.ldq);
            if (j < na) srow[j - base] = valid ? qn : 0.0;
          }
        }
      }
    };
    // first half: columns 0..31 (the augmented v, f when they fall there)
    sweep(0, 32, 0);
    if (a.naug > 0 && kk < 32) srow[kk] = av;
    if (a.naug > 1 && kk + 1 < 32) srow[kk + 1] = af;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double h0[16], h1[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 4 * q + lk;
      h0[q] = stage[r * kHalfStride + li];
      h1[q] = stage[r * kHalfStride + 16 + li];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(h0[q], h0[q], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(h1[q], h0[q], acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(h1[q], h1[q], acc[2], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // second half: columns 32 .. na-1
    sweep(32, 64, 32);
    if (a.naug > 0 && kk >= 32) srow[kk - 32] = av;
    if (a.naug > 1 && kk + 1 >= 32) srow[kk - 31] = af;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 4 * q + lk;
      const double v2 = live2 ? stage[r * kHalfStride + li] : 0.0;
      const double v3 = live3 ? stage[r * kHalfStride + 16 + li] : 0.0;
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(v2, h0[q], acc[3], 0, 0, 0);
      acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(v2, h1[q], acc[4], 0, 0, 0);
      acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(v2, v2, acc[5], 0, 0, 0);
      if (blk3) {
        acc[6] = __builtin_amdgcn_mfma_f64_16x16x4f64(v3, h0[q], acc[6], 0, 0, 0);
        acc[7] = __builtin_amdgcn_mfma_f64_16x16x4f64(v3, h1[q], acc[7], 0, 0, 0);
        acc[8] = __builtin_amdgcn_mfma_f64_16x16x4f64(v3, v2, acc[8], 0, 0, 0);
        acc[9] = __builtin_amdgcn_mfma_f64_16x16x4f64(v3, v3, acc[9], 0, 0, 0);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Write this wave's Gram accumulators as pair sums accw[a(a-1)/2 + b],
// b < a < kk.
template <int KMAX>
__device__ inline void gram_store(const v4d (&acc)[GramShape<KMAX>::NBP], double* accw, int kk) {
  using S = GramShape<KMAX>;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  int p = 0;
#pragma unroll
  for (int bi = 0; bi < S::NB; ++bi)
#pragma unroll
    for (int bj = 0; bj <= bi; ++bj, ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ia = bi * 16 + lk + 4 * r, ib = bj * 16 + li;
        if (ia > ib && ia < kk) accw[ia * (ia - 1) / 2 + ib] = acc[p][r];
      }
}

// ---------------------------------------------------------------------------
// elementwise passes
// ---------------------------------------------------------------------------

// (A u)_p, A the (2 dim + 1)-point Dirichlet Laplacian on an s^dim grid
// (x fastest) scaled by ih2 = 1/h^2.
__device__ __forceinline__ double lap_point(const double* __restrict__ u, int dim, int64_t s,
                                            double ih2, int64_t p) {
  const int64_t ix = p % s;
  const double up = u[p];
  double nb = 0.0;
  if (ix > 0) nb += u[p - 1];
  if (ix < s - 1) nb += u[p + 1];
  if (dim >= 2) {
    const int64_t iy = (p / s) % s;
    if (iy > 0) nb += u[p - s];
    if (iy < s - 1) nb += u[p + s];
  }
  if (dim >= 3) {
    const int64_t s2 = s * s, iz = p / s2;
    if (iz > 0) nb += u[p - s2];
    if (iz < s - 1) nb += u[p + s2];
  }
  return (2.0 * dim * up - nb) * ih2;
}

// G(u)_p = u_p - omega ((A u)_p + c u_p^3 - f_p), A the (2 dim + 1)-point
// Dirichlet Laplacian on an s^dim grid (x fastest) scaled by ih2 = 1/h^2.
__device__ __forceinline__ double stencil_point(const double* __restrict__ u,
                                                const double* __restrict__ f, int dim,
                                                int64_t s, double ih2, double omega, double c,
                                                int64_t p) {
  const int64_t ix = p % s;
  const double up = u[p];
  double nb = 0.0;
  if (ix > 0) nb += u[p - 1];
  if (ix < s - 1) nb += u[p + 1];
  if (dim >= 2) {
    const int64_t iy = (p / s) % s;
    if (iy > 0) nb += u[p - s];
    if (iy < s - 1) nb += u[p + s];
  }
  if (dim >= 3) {
    const int64_t s2 = s * s, iz = p / s2;
    if (iz > 0) nb += u[p - s2];
    if (iz < s - 1) nb += u[p + s2];
  }
  const double au = (2.0 * dim * up - nb) * ih2;
  return up - omega * (au + c * up * up * up - f[p]);
}

// out = in / d over pairs p = t0 * kWG + tid, stride ts * kWG (and the odd tail).
__device__ inline void scale_body(const double* in, double* out, int64_t n, double d,
                                  int64_t t0, int64_t ts) {
  const int64_t npair = n / 2;
  const double2* in2 = reinterpret_cast<const double2*>(in);
  double2* out2 = reinterpret_cast<double2*>(out);
  for (int64_t r = t0 * kWG + threadIdx.x; r < npair; r += ts * kWG) {
    const f64x2 v = ld2v(in2 + r);
#if AA_NT_STORE
    f64x2 o;
    o.x = v.x / d;
    o.y = v.y / d;
    __builtin_nontemporal_store(o, reinterpret_cast<f64x2*>(out2 + r));
#else
    out2[r] = make_double2(v.x / d, v.y / d);
#endif
  }
  if (t0 == 0 && threadIdx.x == 0 && (n & 1)) out[n - 1] = in[n - 1] / d;
}

// i >= 1 (Alg. 1): f = g - x; Delta f = f - f_prev -> W; Delta g = g - g_prev
// -> ring slot; f_prev <- f; g_prev <- g; acc_w[0] += ||f||^2.
// i == 0: f_prev = g - x, g_prev = g, x_next = g; acc_w[0..1] += ||f||^2.
__device__ inline void history_body(const HistArgs& a, int64_t t0, int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  double sff = 0.0;  // this lane's share of ||f||^2 over all its tiles
  for_tiles(a.n, t0, ts, [&](int64_t b2, auto full) {
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
    sff += dot2(f, f);
  });
  const double p = wave_sum(sff);
  if (lane == 0) {
    acc[0] += p;
    acc[1] += p;  // first step: x_1 - x_0 = f_0
  }
}

// Alg. 1: x_{i+1} = g_i - sum_j gamma_j Delta g_{i-m_i+j}; acc_w[0] += ||x_{i+1}-x_i||^2.
__device__ inline void xupdate_coefs(const XupdArgs& a, double* s_g, int* s_slot) {
  for (int j = threadIdx.x; j < a.mi; j += blockDim.x) {
    s_g[j] = a.gamma[j];
    s_slot[j] = (a.slot0 + j) % a.m;
  }
}

__device__ inline void xupdate_body(const XupdArgs& a, const double* s_g, const int* s_slot,
                                    int64_t t0, int64_t ts, double* acc) {
  const int lane = threadIdx.x & 63;
  double sdx = 0.0;  // this lane's share of ||x_{i+1} - x_i||^2
  for_tiles(a.n, t0, ts, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 gv[kPairs], xv[kPairs], sum[kPairs];
    ld2<F>(gv, a.g, b2, a.n);
    ld2<F>(xv, a.x, b2, a.n);
    zero2(sum);
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
        if (g0 + c < a.mi) axpy2(sum, d[c], s_g[g0 + c]);
    }
    double d2 = 0.0;
#pragma unroll
    for (int i = 0; i < kPairs; ++i) {
      const double2 xn = make_double2(gv[i].x - sum[i].x, gv[i].y - sum[i].y);
      const double dx = xn.x - xv[i].x, dy = xn.y - xv[i].y;
      d2 = fma(dx, dx, d2);
      d2 = fma(dy, dy, d2);
      gv[i] = xn;
    }
    st2<F>(gv, a.x_next, b2, a.n);
    sdx += d2;
  });
  const double p = wave_sum(sdx);
  if (lane == 0) acc[0] += p;
}

}  // namespace aa
