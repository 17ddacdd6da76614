// aa_batch.hip -- one Anderson-acceleration iteration per workgroup.
//
// Used two ways:
//  * batched AA: thousands of independent instances (uneven n and window m)
//    advance one iteration each in a single persistent launch.  Workgroups
//    pull instances from an atomic work counter in a fixed order (largest
//    n * m first, so the long instances start early); an instance is owned by
//    one workgroup for the whole iteration, so every "Sync" of the paper is a
//    workgroup barrier plus an LDS reduction.  Converged instances (relative
//    residual below tol) are skipped.
//  * the fused single-instance step for small n: the same code with one
//    instance, the caller's x / G(x) / x_next, and the host's iteration
//    counters, replacing ~30 small launches by one.
// The passes are the bodies of aa_passes.h with tiles 0, 1, 2, ... (one
// workgroup); the dense tails are the same as in the grid path.
#include <math.h>

// Row pairs per lane per tile in this translation unit.  One workgroup walks
// an instance's whole vectors, waiting on every tile's loads in turn, so
// longer tiles (fewer waits) pay here: four pairs instead of the grid passes'
// two took the one-instance step from 84 to 77 us (n = 4096, m = 5) and from
// 654 to 564 us (n = 13824, m = 20).  Only device code sees the value (no
// host code shares it), so the two translation units may differ.
//
// The file is compiled twice: as itself (four row pairs, namespace aa::p4,
// with the host helpers), and through aa_batch_p2.hip with two row pairs
// (namespace aa::p2, AA_BATCH_SECONDARY): the batch schedule autotuner
// chooses the tiling at run time.
#ifndef AA_PAIRS
#define AA_PAIRS 4
#endif
#ifndef AA_BATCH_SECONDARY
#define AA_BATCH_SECONDARY 0
#endif
#include "aa_passes.h"

namespace aa {
#if AA_BATCH_SECONDARY
namespace p2 {
#else
namespace p4 {
#endif

__device__ __forceinline__ Tail mk_tail(int op, int k) {
  Tail t{};
  t.op = op;
  t.k = k;
  return t;
}

template <int KB, bool GRAM>
struct BatchLds {
  static constexpr int KG = KB < 16 ? 16 : KB;          // Gram block bucket
  static constexpr int NACC = 3 * KB + 4;                // per-wave accumulators
  static constexpr int NPG = GRAM ? GramShape<KG>::NP : 1;
  static constexpr int NRED = NACC > NPG ? NACC : NPG;
  double acc[kWaves * NACC];
  double red[NRED];
  double c1[kMaxCols], c2[kMaxCols], cs[kMaxCols];
  double gc[KG], gs[KG];
  double sg[kMaxCols];
  int sslot[kMaxCols];
};

// Dynamic LDS of the batched kernel: the Givens scratch (KB x KB), which is
// dead once the rotations exist, then (ICWY) the Gram staging of the rotated
// rows, sized on the host for the largest window of the batch
// (max(KB^2, gram_lds_doubles(m_max - 1)) doubles).
extern __shared__ double batch_dyn[];

// Zero the accumulators, run body(this wave's accumulators), combine the
// waves into red[0:nred], run the dense tail.  All threads call.
template <class L, class Body>
__device__ __forceinline__ void wg_pass(const Small& sm, const Tail& t, int nred, L& lds,
                                        Body&& body) {
  constexpr int S = L::NACC;
  lds_zero(lds.acc, kWaves * S);
  __syncthreads();
  body(lds.acc + (threadIdx.x >> 6) * S);
  __syncthreads();
  for (int c = threadIdx.x; c < nred; c += kWG) {
    double s = lds.acc[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds.acc[w * S + c];
    lds.red[c] = s;
  }
  __syncthreads();
  run_tail(sm, t, lds.red);
  __syncthreads();
}

// w -> w / R_kk (the normalization that ends every QRAdd).
template <class L>
__device__ __forceinline__ void wg_scale(const Small& sm, int k, const double* in, double* out,
                                         int64_t n) {
  scale_body(in, out, n, sm.R[k + (size_t)k * sm.cap], 0, 1);
  __syncthreads();
}

// QRAdd (Alg. 2 with Algs. 3-6) of v as column k; k columns present.  With
// f (not MGS, k >= 1) the passes also form c = Q^T f and the norm pass's tail
// solves R gamma = c (as AA_FUSE_RHS on the grid path).  first_done: the
// first pass's reduction and tail already ran (fused with QRDelete).
template <int KB, class L>
__device__ void wg_qr_add(const BInst& I, int variant, unsigned flags, int k, const double* v,
                          L& lds, const double* f = nullptr, bool first_done = false) {
  const Small& sm = I.sm;
  const bool fuse = f != nullptr && k >= 1 && variant != AA_MGS;
  double* slotk = I.Q + (int64_t)k * I.ld;
  double* Rcol = sm.R + (size_t)k * sm.cap;
  DotsArgs d{I.Q, I.ld, I.n, v, 0, nullptr, 0, 0};
  UpdArgs u{};
  u.Q = I.Q; u.ldq = I.ld; u.n = I.n; u.Qw = I.Q; u.dotcol = -1; u.dcgs2_p = -1;
  Tail tn = mk_tail(TAIL_NORM, k);
  tn.idx = 0;
  auto dots = [&](const DotsArgs& a, const Tail& t) {
    if (first_done) return;
    wg_pass(sm, t, a.nx + a.ny + a.nz + (a.xx ? 1 : 0), lds,
            [&](double* acc) { dots_body(a, 0, 1, acc); });
  };
  auto update = [&](const UpdArgs& a, const Tail& t) {
    update_coefs(a, lds.c1, lds.c2, lds.cs);
    wg_pass(sm, t, update_nred(a), lds,
            [&](double* acc) { update_body(a, lds.c1, lds.c2, lds.cs, 0, 1, acc); });
  };
  if (fuse) {
    tn.rhs = 1;
    d.z = f;
    d.nz = k;
  }
  if (k == 0) {
    d.xx = 1;
    dots(d, tn);
    wg_scale<L>(sm, 0, v, slotk, I.n);
    return;
  }
  switch (variant) {
    case AA_MGS: {
      Tail t0 = mk_tail(TAIL_MGS_R, k);
      t0.row = 0;
      d.nx = 1;
      dots(d, t0);
      const double* cur = v;
      for (int j = 1; j < k; ++j) {
        UpdArgs uj = u;
        uj.v = cur; uj.out = I.W; uj.j0 = j - 1; uj.nc = 1; uj.c1 = Rcol; uj.dotcol = j;
        Tail tj = mk_tail(TAIL_MGS_R, k);
        tj.row = j;
        update(uj, tj);
        cur = I.W;
      }
      UpdArgs uk = u;
      uk.v = cur; uk.out = slotk; uk.j0 = k - 1; uk.nc = 1; uk.c1 = Rcol; uk.nrm = 1;
      update(uk, tn);
      break;
    }
    case AA_CGS2: {
      d.nx = k;
      Tail ts = mk_tail(TAIL_CGS2_S, k);
      ts.rhs = fuse ? 1 : 0;
      ts.zoff = k;
      dots(d, ts);
      for (int j = threadIdx.x; j < KB; j += kWG) lds.cs[j] = (j < k) ? sm.coef0[j] : 0.0;
      Cgs2bArgs b{I.Q, I.ld, I.n, v, k, sm.coef0};
      wg_pass(sm, mk_tail(TAIL_CGS2_Z, k), k, lds, [&](double* acc) {
        if constexpr (KB <= 8)
          cgs2b_reg_body<8>(b, lds.cs, 0, 1, acc);
        else
          cgs2b_stream_body(b, lds.cs, 0, 1, acc);
      });
      UpdArgs uc = u;
      uc.v = v; uc.out = slotk; uc.j0 = 0; uc.nc = k; uc.c1 = sm.coef0; uc.c2 = sm.coef1;
      uc.nrm = 1;
      uc.rhsv = fuse ? f : nullptr;
      update(uc, tn);
      break;
    }
    case AA_ICWY: {
      d.nx = k;
      d.y = I.Q + (int64_t)(k - 1) * I.ld;
      d.ny = k - 1;
      Tail ti = mk_tail(TAIL_ICWY, k);
      ti.rhs = fuse ? 1 : 0;
      ti.zoff = 2 * k - 1;
      dots(d, ti);
      UpdArgs ub = u;
      ub.v = v; ub.out = slotk; ub.j0 = 0; ub.nc = k; ub.c1 = sm.coef0; ub.nrm = 1;
      ub.rhsv = fuse ? f : nullptr;
      update(ub, tn);
      break;
    }
    default: {  // AA_DCGS2
      const int m_i = k + 1;
      const bool reorth = (flags & AA_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
      d.nx = k;
      d.y = I.Q + (int64_t)(k - 1) * I.ld;
      d.ny = reorth ? k - 1 : 0;
      Tail ta = mk_tail(TAIL_DCGS2, k);
      ta.reorth = reorth;
      ta.literal = (flags & AA_DCGS2_LITERAL) ? 1 : 0;
      ta.rhs = fuse ? 1 : 0;
      ta.zoff = k + d.ny;
      dots(d, ta);
      UpdArgs ub = u;
      ub.v = v; ub.out = slotk; ub.c1 = Rcol; ub.nrm = 1;
      ub.rhsv = fuse ? f : nullptr;
      if (reorth) {
        ub.dcgs2_p = k - 1; ub.reorth = 1; ub.s = sm.coef1; ub.j0 = 0; ub.nc = k - 1;
      } else {
        ub.j0 = 0; ub.nc = k;
      }
      update(ub, tn);
      break;
    }
  }
  wg_scale<L>(sm, k, slotk, slotk, I.n);
}

// Rotation sweep of r plus the strict lower Gram of its staged columns
// (gram_cols(r): the rotated ones, minus the last with drop_last, then v and
// f), summed over the workgroup into red[a (a - 1) / 2 + b], b < a.  Up to 8
// rotated-or-staged columns on the vector units (rotate_gram_small_body: a
// 16 x 16 MFMA block would spend 256 multiply-adds per row on them), wider
// windows on the matrix cores (rotate_gram_body).
template <int KG>
__device__ void wg_rotate_gram(const RotArgs& r, const double* gc, const double* gs, double* red) {
  const int na = gram_cols(r), np = na * (na - 1) / 2;
  if (r.k - 1 + r.naug <= 8) {
    double acc[32];
    rotate_gram_small_body<8>(r, gc, gs, 0, 1, acc);
    const double v = multi_reduce<32>(acc);  // lane l < 32: pair l over the wave
    const int lane = threadIdx.x & 63;
    if (lane < np) batch_dyn[(threadIdx.x >> 6) * np + lane] = v;
  } else {
    using S = GramShape<KG>;
    v4d acc[S::NBP];
    rotate_gram_body<KG>(r, gc, gs, 0, 1, batch_dyn, gram_stride(na), acc);
    __syncthreads();
    gram_store<KG>(acc, batch_dyn + (threadIdx.x >> 6) * np, na);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < np; c += kWG) {
    double s = batch_dyn[c];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += batch_dyn[w * np + c];
    red[c] = s;
  }
  __syncthreads();
}

// QRDelete (Alg. 2): Givens rotations from R, one sweep over Q; ICWY also
// refreshes T (Gram of the rotated columns).  The QRAdd that follows in the
// same iteration recomputes the last row of T from its first reduction
// (Alg. 4) before anything reads it, so the Gram leaves the last rotated
// column out.
template <int KB, bool GRAM, class L>
__device__ void wg_qr_delete(const BInst& I, int variant, int k, L& lds) {
  const Small& sm = I.sm;
  if (k <= 1) return;
  givens_body(sm, k, batch_dyn);
  __syncthreads();
  RotArgs r{I.Q, I.ld, I.n, k, sm.givens, 0};
  givens_coefs(r, sm.cap, lds.gc, lds.gs, L::KG);
  __syncthreads();
  if constexpr (GRAM) {
    if (variant == AA_ICWY) {
      r.gram = 1;
      r.drop_last = 1;
      wg_rotate_gram<L::KG>(r, lds.gc, lds.gs, lds.red);
      run_tail(sm, mk_tail(TAIL_GRAM, gram_cols(r)), lds.red);
      __syncthreads();
      return;
    }
  }
  rotate_body(r, lds.gc, lds.gs, 0, 1);
  __syncthreads();
}

// out = G(u) over one instance by one workgroup.  Each thread evaluates four
// points per round with all their loads issued before any result is stored
// (the pointers do not alias), and 32-bit index arithmetic (an instance has
// far fewer than 2^31 points): the plain per-point loop waits out one memory
// latency per point.
__device__ __forceinline__ void wg_stencil(const double* __restrict__ u,
                                           const double* __restrict__ f,
                                           double* __restrict__ out, int dim, int64_t s64,
                                           double ih2, double omega, double c, int64_t n64) {
  if (n64 >= (int64_t)1 << 30) {
    for (int64_t p = threadIdx.x; p < n64; p += kWG)
      out[p] = stencil_point(u, f, dim, s64, ih2, omega, c, p);
    return;
  }
  constexpr int U = 4;
  const int n = (int)n64, s = (int)s64, s2 = s * s;
  for (int p0 = threadIdx.x; p0 < n; p0 += U * kWG) {
    double up[U], nb[U], fp[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int p = p0 + q * kWG;
      up[q] = nb[q] = fp[q] = 0.0;
      if (p < n) {
        const int ix = p % s;
        up[q] = u[p];
        fp[q] = f[p];
        double a = 0.0;
        if (ix > 0) a += u[p - 1];
        if (ix < s - 1) a += u[p + 1];
        if (dim >= 2) {
          const int iy = (p / s) % s;
          if (iy > 0) a += u[p - s];
          if (iy < s - 1) a += u[p + s];
        }
        if (dim >= 3) {
          const int iz = p / s2;
          if (iz > 0) a += u[p - s2];
          if (iz < s - 1) a += u[p + s2];
        }
        nb[q] = a;
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int p = p0 + q * kWG;
      if (p < n) {
        const double au = (2.0 * dim * up[q] - nb[q]) * ih2;
        out[p] = up[q] - omega * (au + c * up[q] * up[q] * up[q] - fp[q]);
      }
    }
  }
}

// Whether QRDelete with k columns can share its pass with the QRAdd's first
// (AA_FUSE_DELETE, not MGS; the staged [Q v (f)] must fit the Gram bucket).
template <bool GRAM, class L>
__device__ __forceinline__ bool delete_fusable(const BatchArgs& b, int k, bool rhs) {
  if constexpr (!GRAM) {
    return false;
  } else {
    return (b.flags & AA_FUSE_DELETE) && b.variant != AA_MGS && k >= 2 &&
           k - 1 + (rhs ? 2 : 1) <= L::KG;
  }
}

// QRDelete fused with the first pass of the QRAdd of v (AA_FUSE_DELETE): the
// rotation stages v (and f) beside the rotated rows, one Gram of [Q v (f)]
// on the matrix cores gives ICWY's T refresh and every block dot product of
// the QRAdd's first pass; they are laid out as that pass would have reduced
// them and its tail runs.  k columns present on entry (k - 1 after).
template <int KB, bool GRAM, class L>
__device__ void wg_delete_first_pass(const BInst& I, int variant, unsigned flags, int k,
                                     const double* v, const double* f, L& lds) {
  if constexpr (GRAM) {
    const Small& sm = I.sm;
    givens_body(sm, k, batch_dyn);
    __syncthreads();
    const int naug = f ? 2 : 1;
    RotArgs r{I.Q, I.ld, I.n, k, sm.givens, 1, v, f, naug};
    givens_coefs(r, sm.cap, lds.gc, lds.gs, L::KG);
    __syncthreads();
    const int kk = k - 1;
    wg_rotate_gram<L::KG>(r, lds.gc, lds.gs, lds.red);
    if (variant == AA_ICWY) {
      run_tail(sm, mk_tail(TAIL_GRAM, kk), lds.red);
      __syncthreads();
    }
    // the first pass's tail and layout for kk columns (as wg_qr_add builds them)
    Tail t = mk_tail(TAIL_ICWY, kk);
    t.rhs = f ? 1 : 0;
    bool row = true;
    if (variant == AA_CGS2) {
      t.op = TAIL_CGS2_S;
      t.zoff = kk;
      row = false;
    } else if (variant == AA_ICWY) {
      t.zoff = 2 * kk - 1;
    } else {
      const int m_i = kk + 1;
      t.op = TAIL_DCGS2;
      t.reorth = (flags & AA_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
      t.literal = (flags & AA_DCGS2_LITERAL) ? 1 : 0;
      t.zoff = kk + (t.reorth ? kk - 1 : 0);
      row = t.reorth != 0;
    }
    const int pv = kk * (kk - 1) / 2, pf = (kk + 1) * kk / 2, prow = (kk - 1) * (kk - 2) / 2;
    double* red2 = lds.acc;  // free between passes
    for (int b2 = threadIdx.x; b2 < kk; b2 += kWG) {
      red2[b2] = lds.red[pv + b2];
      if (row && b2 < kk - 1) red2[kk + b2] = lds.red[prow + b2];
      if (f) red2[t.zoff + b2] = lds.red[pf + b2];
    }
    __syncthreads();
    run_tail(sm, t, red2);
    __syncthreads();
  }
}

// dst = src over n values by the whole workgroup (nothing when they alias).
__device__ void wg_copy(const double* src, double* dst, int64_t n) {
  if (src != dst)
    for (int64_t r = threadIdx.x; r < n; r += kWG) dst[r] = src[r];
  __syncthreads();
}

// Front of one iteration of Alg. 1 for one instance (every thread of the
// workgroup): G, history formation, the stopping test, QRDelete, QRAdd and
// R gamma = Q^T f_i.  Returns false when the iteration ends here (the first
// step x_1 = G(x_0), or the instance stopped).
template <int KB, bool GRAM, class L>
__device__ bool wg_front(const BatchArgs& b, const BInst& I, BState& st, L& lds,
                         const double* x, double* xn, const double* g) {
  const int tid = threadIdx.x;
  const Small& sm = I.sm;
  if (!b.og && I.dim > 0 && !st.g_valid) {
    const double ih2 = 1.0 / (I.h * I.h);
    wg_stencil(x, I.f, I.g, I.dim, I.s, ih2, I.omega, I.c, I.n);
    __syncthreads();
    st.g_evals += 1;
  }
  st.g_valid = 0;
  const int64_t it = st.iter;
  if (it == 0) {
    // Alg. 1 before the loop: x_1 = G(x_0), f_0 = G(x_0) - x_0
    HistArgs h{x, g, I.W, I.f_prev, I.g_prev, nullptr, xn, I.n, 1};
    wg_pass(sm, mk_tail(TAIL_FIRST, 0), 2, lds, [&](double* acc) { history_body(h, 0, 1, acc); });
    st.iter = 1;
    st.m_i = 0;
    st.res_norm = st.res0_norm = sqrt(sm.scal[S_RES]);
    return false;
  }
  const int m = I.m;
  const int m_i = (int)(it < m ? it : m);
  const int slot = (int)((it - 1) % m);
  HistArgs h{x, g, I.W, I.f_prev, I.g_prev, I.ring + (int64_t)slot * I.ld, nullptr, I.n, 0};
  Tail tr = mk_tail(TAIL_RES, st.k);
  if (b.ov_iter >= 0) {  // fused single-instance step: the context's stopping test
    tr.stop_mode = b.stop_mode;
    tr.stop_tol = b.stop_tol;
    tr.m_i = st.m_i;
  }
  wg_pass(sm, tr, 1, lds, [&](double* acc) { history_body(h, 0, 1, acc); });
  if (b.ov_iter >= 0 && sm.stop && sm.stop->done != 0) {
    // the test held at the start of this iteration: x_next = x_i
    wg_copy(x, xn, I.n);
    return false;
  }
  const double res = sqrt(sm.scal[S_RES]);
  st.res_norm = res;
  st.status = *sm.status;
  if (b.ov_iter < 0 && (res <= b.tol * st.res0_norm || it >= b.max_iter || st.status != AA_OK)) {
    st.active = 0;
    st.conv_iter = it;
    return false;
  }
  int k = st.k;
  // AA_FUSE_RHS: c = Q^T f_i inside the QRAdd passes (not MGS, not the first add)
  const double* fr =
      ((b.flags & AA_FUSE_RHS) && b.variant != AA_MGS && I.m + 1 <= 64) ? I.f_prev : nullptr;
  const bool rhs_folded = fr != nullptr && (it > m ? k - 1 : k) >= 1;
  if (it > m) {
    if (delete_fusable<GRAM, L>(b, k, fr != nullptr)) {
      wg_delete_first_pass<KB, GRAM>(I, b.variant, b.flags, k, I.W, fr, lds);
      k -= 1;
      wg_qr_add<KB>(I, b.variant, b.flags, k, I.W, lds, fr, true);
    } else {
      wg_qr_delete<KB, GRAM>(I, b.variant, k, lds);
      k -= 1;
      wg_qr_add<KB>(I, b.variant, b.flags, k, I.W, lds, fr);
    }
  } else {
    wg_qr_add<KB>(I, b.variant, b.flags, k, I.W, lds, fr);
  }
  k += 1;
  if (!rhs_folded) {
    DotsArgs d{I.Q, I.ld, I.n, I.f_prev, k, nullptr, 0, 0};
    wg_pass(sm, mk_tail(TAIL_RHS, k), k, lds, [&](double* acc) { dots_body(d, 0, 1, acc); });
  }
  st.k = k;
  st.m_i = m_i;
  st.status = *sm.status;
  return true;
}

// x_{i+1} = G(x_i) - sum_j gamma_j Delta g_{i-m_i+j}  (the plain AA update).
template <class L>
__device__ void wg_plain_update(const BInst& I, const BState& st, L& lds, const double* x,
                                double* xn, const double* g) {
  const int64_t it = st.iter;
  const int m = I.m, m_i = st.m_i;
  XupdArgs xa{I.ring, I.ld, m, (int)((it - m_i) % m), m_i, g, x, xn, I.n, I.sm.gamma};
  xupdate_coefs(xa, lds.sg, lds.sslot);
  wg_pass(I.sm, mk_tail(TAIL_STEP, 0), 1, lds,
          [&](double* acc) { xupdate_body(xa, lds.sg, lds.sslot, 0, 1, acc); });
}

// Network features of the current state: upper triangle of R over a 20-column
// window (row-major, a <= b), then c = Q^T f_i, both divided by ||f_i||.
__device__ void write_features(const BInst& I, const BState& st, float* row, bool live) {
  const Small& sm = I.sm;
  const int k = st.k;
  const double inv = live ? 1.0 / st.res_norm : 0.0;
  for (int t = threadIdx.x; t < kFeat; t += kWG) {
    double v = 0.0;
    if (live) {
      if (t < kWin * (kWin + 1) / 2) {
        int a = 0, rem = t;
        while (rem >= kWin - a) {
          rem -= kWin - a;
          ++a;
        }
        const int bcol = a + rem;
        if (bcol < k) v = sm.R[a + (size_t)bcol * sm.cap];
      } else {
        const int j = t - kWin * (kWin + 1) / 2;
        if (j < k) v = sm.coef1[j];
      }
    }
    row[t] = (float)(v * inv);
  }
}

// The learned candidate: gamma' = gamma + delta gamma (first m_i outputs),
// beta = sigmoid(o_20), w = R gamma', x_c = g - G_i gamma' - (1 - beta)(f_i - Q w)
// into I.xc; then G(x_c) into I.gc.  Leaves gamma' in lds.c1, w in lds.c2,
// slot order in lds.sslot; returns beta.
template <class L>
__device__ double wg_candidate(const BatchArgs& b, const BInst& I, const BState& st, L& lds,
                               const double* g, int row_index) {
  const Small& sm = I.sm;
  const int m = I.m, m_i = st.m_i, k = st.k;
  const float* o = b.out + (size_t)row_index * kOuts;
  for (int j = threadIdx.x; j < m_i; j += kWG) {
    lds.c1[j] = sm.gamma[j] + (double)o[j];
    lds.sslot[j] = (int)((st.iter - m_i + j) % m);
  }
  __syncthreads();
  for (int a = threadIdx.x; a < k; a += kWG) {
    double acc = 0.0;
    for (int c = a; c < k; ++c) acc += sm.R[a + (size_t)c * sm.cap] * lds.c1[c];
    lds.c2[a] = acc;
  }
  __syncthreads();
  const double beta = 1.0 / (1.0 + exp(-(double)o[kWin]));
  const double omb = 1.0 - beta;
  for_tiles(I.n, 0, 1, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 gv[kPairs], fv[kPairs], ar[kPairs], aq[kPairs], dummy[kPairs];
    ld2<F>(gv, g, b2, I.n);
    ld2<F>(fv, I.f_prev, b2, I.n);
    zero2(ar);
    zero2(aq);
    for (int j = 0; j < m_i; ++j) {
      double2 d[kPairs];
      ld2<F>(d, I.ring + (int64_t)lds.sslot[j] * I.ld, b2, I.n);
      axpy2(ar, d, lds.c1[j]);
    }
    combine_cols<F>(I.Q, I.ld, b2, I.n, 0, k, lds.c2, nullptr, aq, dummy);
#pragma unroll
    for (int i = 0; i < kPairs; ++i) {
      gv[i].x = (gv[i].x - ar[i].x) - omb * (fv[i].x - aq[i].x);
      gv[i].y = (gv[i].y - ar[i].y) - omb * (fv[i].y - aq[i].y);
    }
    st2<F>(gv, I.xc, b2, I.n);
  });
  __syncthreads();
  const double ih2 = 1.0 / (I.h * I.h);
  wg_stencil(I.xc, I.f, I.gc, I.dim, I.s, ih2, I.omega, I.c, I.n);
  __syncthreads();
  return beta;
}

// ||G(x_c) - x_c||^2; with store_r the residual replaces G(x_c) in I.gc.
template <class L>
__device__ double wg_cand_residual(const BInst& I, L& lds, bool store_r) {
  wg_pass(I.sm, mk_tail(TAIL_NONE, 0), 1, lds, [&](double* acc) {
    const int lane = threadIdx.x & 63;
    for_tiles(I.n, 0, 1, [&](int64_t b2, auto full) {
      constexpr bool F = decltype(full)::value;
      double2 gc[kPairs], xc[kPairs];
      ld2<F>(gc, I.gc, b2, I.n);
      ld2<F>(xc, I.xc, b2, I.n);
#pragma unroll
      for (int i = 0; i < kPairs; ++i) gc[i] = make_double2(gc[i].x - xc[i].x, gc[i].y - xc[i].y);
      if (store_r) st2<F>(gc, I.gc, b2, I.n);
      const double p = wave_sum(dot2(gc, gc));
      if (lane == 0) acc[0] += p;
    });
  });
  return lds.red[0];
}

// Accept the candidate: x <- x_c, G(x) <- G(x_c) (known for the next iteration).
__device__ void wg_accept(const BInst& I, double* xn) {
  for_tiles(I.n, 0, 1, [&](int64_t b2, auto full) {
    constexpr bool F = decltype(full)::value;
    double2 v[kPairs];
    ld2<F>(v, I.xc, b2, I.n);
    st2<F>(v, xn, b2, I.n);
    ld2<F>(v, I.gc, b2, I.n);
    st2<F>(v, I.g, b2, I.n);
  });
  __syncthreads();
}

// Training: gradient of L = log(||r||^2 / ||f_i||^2), r = G(x_c) - x_c, with
// respect to the network outputs.  dL/dx_c = (2 / ||r||^2) J_f^T r with
// J_f = J - I = -omega (A + 3 c diag(x_c^2)) symmetric; then
// dL/dgamma' = -G_i^T v + (1 - beta) R^T (Q^T v), dL/dbeta = f_i^T v - w^T (Q^T v).
template <class L>
__device__ void wg_train_grad(const BatchArgs& b, const BInst& I, BState& st, L& lds, double beta,
                              double r2, int row_index) {
  const Small& sm = I.sm;
  const int m_i = st.m_i, k = st.k;
  const double res = st.res_norm;
  st.loss = log(r2 / (res * res));
  const double ih2 = 1.0 / (I.h * I.h);
  const double sc = 2.0 / r2;
  for (int64_t p = threadIdx.x; p < I.n; p += kWG) {
    const double xc = I.xc[p], rp = I.gc[p];
    const double jr = -I.omega * (lap_point(I.gc, I.dim, I.s, ih2, p) + 3.0 * I.c * xc * xc * rp);
    I.xc[p] = sc * jr;  // v overwrites x_c (each point reads its own x_c first)
  }
  __syncthreads();
  // ring^T v over the m_i slots in use (contiguous 0..m_i-1), Q^T v, f^T v
  DotsArgs dr{I.ring, I.ld, I.n, I.xc, m_i, nullptr, 0, 0};
  wg_pass(sm, mk_tail(TAIL_NONE, 0), m_i, lds, [&](double* acc) { dots_body(dr, 0, 1, acc); });
  for (int j = threadIdx.x; j < m_i; j += kWG) lds.cs[j] = lds.red[j];  // by slot
  DotsArgs dq{I.Q, I.ld, I.n, I.xc, k, I.f_prev, 0, 0};
  wg_pass(sm, mk_tail(TAIL_NONE, 0), k, lds, [&](double* acc) { dots_body(dq, 0, 1, acc); });
  for (int j = threadIdx.x; j < k; j += kWG) lds.sg[j] = lds.red[j];   // Q^T v
  wg_pass(sm, mk_tail(TAIL_NONE, 0), 1, lds, [&](double* acc) {
    const int lane = threadIdx.x & 63;
    for_tiles(I.n, 0, 1, [&](int64_t b2, auto full) {
      constexpr bool F = decltype(full)::value;
      double2 fv[kPairs], vv[kPairs];
      ld2<F>(fv, I.f_prev, b2, I.n);
      ld2<F>(vv, I.xc, b2, I.n);
      const double p = wave_sum(dot2(fv, vv));
      if (lane == 0) acc[0] += p;
    });
  });
  const double fv = lds.red[0];
  float* drow = b.dout + (size_t)row_index * kOuts;
  const double omb = 1.0 - beta;
  for (int j = threadIdx.x; j < kWin; j += kWG) {
    double d = 0.0;
    if (j < m_i) {
      double rtb = 0.0;
      for (int a = 0; a <= j; ++a) rtb += sm.R[a + (size_t)j * sm.cap] * lds.sg[a];
      d = -lds.cs[lds.sslot[j]] + omb * rtb;
    }
    drow[j] = (float)(d * b.dscale);
  }
  if (threadIdx.x == 0) {
    double wb = 0.0;
    for (int a = 0; a < k; ++a) wb += lds.c2[a] * lds.sg[a];
    drow[kWin] = (float)((fv - wb) * beta * (1.0 - beta) * b.dscale);
  }
  __syncthreads();
}

// One unit of work for one instance in the given mode (every thread).
template <int KB, bool GRAM, class L>
__device__ BState wg_instance(const BatchArgs& b, const BInst& I, BState st, L& lds, int j) {
  const double* x = b.ox ? b.ox : I.x;
  double* xn = b.oxn ? b.oxn : I.x;
  const double* g = b.og ? b.og : I.g;
  switch (b.mode) {
    case BM_PHASE_A: {
      const bool more = wg_front<KB, GRAM>(b, I, st, lds, x, xn, g);
      st.pending = more ? 1 : 0;
      write_features(I, st, b.feat + (size_t)j * kFeat, more);
      __syncthreads();
      return st;
    }
    case BM_GUARD:
    case BM_TRAIN: {
      if (!st.pending) {
        if (b.mode == BM_TRAIN)
          for (int t = threadIdx.x; t < kOuts; t += kWG) b.dout[(size_t)j * kOuts + t] = 0.f;
        __syncthreads();
        return st;
      }
      const double beta = wg_candidate(b, I, st, lds, g, j);
      st.g_evals += 1;
      const double r2 = wg_cand_residual(I, lds, b.mode == BM_TRAIN);
      if (b.mode == BM_GUARD && sqrt(r2) < st.res_norm) {
        wg_accept(I, xn);
        st.g_valid = 1;
        st.accepted += 1;
      } else {
        if (b.mode == BM_TRAIN) wg_train_grad(b, I, st, lds, beta, r2, j);
        wg_plain_update(I, st, lds, x, xn, g);
      }
      st.pending = 0;
      st.iter += 1;
      return st;
    }
    default: {
      if (wg_front<KB, GRAM>(b, I, st, lds, x, xn, g)) {
        if (b.ov_iter >= 0 && I.sm.stop && *I.sm.status != AA_OK) {
          // breakdown in this iteration: x_{i+1} = G(x_i), and it ends here
          wg_copy(g, xn, I.n);
          if (threadIdx.x == 0) {
            I.sm.stop->iter = I.sm.stop->cur - 1;
            I.sm.stop->k = st.k;
            I.sm.stop->m_i = st.m_i;
            I.sm.stop->done = AA_STOPPED_BREAKDOWN;
          }
        } else {
          wg_plain_update(I, st, lds, x, xn, g);
        }
        st.iter += 1;
      }
      return st;
    }
  }
}

// At least two waves per SIMD (eight per compute unit): without the bound the
// compiler spends up to 256 registers per lane on this large kernel and only
// one workgroup fits a compute unit; with it (no extra spills) the batched
// iteration of the 4096-instance workload runs 1.5x faster.
template <int KB, bool GRAM>
__global__ __launch_bounds__(kWG, 2) void k_batch(BatchArgs b) {
  using L = BatchLds<KB, GRAM>;
  __shared__ L lds;
  __shared__ int s_idx;
  if (b.ov_iter >= 0) {  // fused single-instance step: host-held counters
    if (aa_stopped(b.inst[0].sm)) {  // the iteration has ended: x_next = x
      wg_copy(b.ox, b.oxn, b.inst[0].n);
      return;
    }
    BState st = b.state[0];
    st.iter = b.ov_iter;
    st.k = b.ov_k;
    st.active = 1;
    const BState out = wg_instance<KB, GRAM>(b, b.inst[0], st, lds, 0);
    if (threadIdx.x == 0) b.state[0] = out;
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(b.counter, 1u);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= b.count) break;
    const int j = b.order[idx];
    if (b.skip && b.skip[j]) continue;  // on the grid-wide passes this iteration
    const BState st = b.state[j];
    if (!st.active && !st.pending) {
      if (b.mode == BM_PHASE_A) write_features(b.inst[j], st, b.feat + (size_t)j * kFeat, false);
      if (b.mode == BM_TRAIN)
        for (int t = threadIdx.x; t < kOuts; t += kWG) b.dout[(size_t)j * kOuts + t] = 0.f;
      continue;
    }
    const BState out = wg_instance<KB, GRAM>(b, b.inst[j], st, lds, j);
    if (threadIdx.x == 0) b.state[j] = out;
    __syncthreads();
  }
}

__global__ void k_batch_reset(unsigned* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// R = 0, T = I, coefficients, Givens, scalars and status cleared; one
// workgroup per instance.
__global__ void k_batch_init(BInst* inst, int count) {
  const int j = blockIdx.x;
  if (j >= count) return;
  const Small sm = inst[j].sm;
  const int cap = sm.cap;
  for (int i = threadIdx.x; i < cap * cap; i += blockDim.x) {
    sm.R[i] = 0.0;
    sm.T[i] = ((i % cap) == (i / cap)) ? 1.0 : 0.0;
  }
  for (int i = threadIdx.x; i < 2 * cap; i += blockDim.x) sm.givens[i] = 0.0;
  for (int i = threadIdx.x; i < cap; i += blockDim.x) {
    sm.coef0[i] = 0.0;
    sm.coef1[i] = 0.0;
    sm.gamma[i] = 0.0;
  }
  if (threadIdx.x < S_COUNT) sm.scal[threadIdx.x] = 0.0;
  if (threadIdx.x == 0) *sm.status = AA_OK;
}

template <bool GRAM>
static hipError_t launch_kb(const BatchArgs& b, int grid, int kb, size_t lds, hipStream_t st) {
  switch (kb) {
    case 8: hipLaunchKernelGGL((k_batch<8, GRAM>), dim3(grid), dim3(kWG), lds, st, b); break;
    case 16: hipLaunchKernelGGL((k_batch<16, GRAM>), dim3(grid), dim3(kWG), lds, st, b); break;
    case 32: hipLaunchKernelGGL((k_batch<32, GRAM>), dim3(grid), dim3(kWG), lds, st, b); break;
    case 64: hipLaunchKernelGGL((k_batch<64, GRAM>), dim3(grid), dim3(kWG), lds, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& b, int grid, int kbucket, bool gram, int stage_cols,
                        hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  if (stage_cols < 0 || stage_cols > (kbucket < 16 ? 16 : kbucket)) return hipErrorInvalidValue;
  int dyn = kbucket * kbucket;
  if (gram && stage_cols > 0 && gram_lds_doubles(stage_cols) > dyn)
    dyn = gram_lds_doubles(stage_cols);
  const size_t lds = sizeof(double) * (size_t)dyn;
  return gram ? launch_kb<true>(b, grid, kbucket, lds, st)
              : launch_kb<false>(b, grid, kbucket, lds, st);
}

}  // namespace p2 / p4

#if !AA_BATCH_SECONDARY
bool batch_needs_gram(int variant, unsigned flags) {
  return variant == AA_ICWY || ((flags & AA_FUSE_DELETE) && variant != AA_MGS);
}

int batch_stage_cols(int mmax, int variant, unsigned flags) {
  if (!batch_needs_gram(variant, flags) || mmax < 2) return 0;
  int cols = mmax - 1;
  if ((flags & AA_FUSE_DELETE) && variant != AA_MGS)
    cols += ((flags & AA_FUSE_RHS) ? 2 : 1);
  const int kb = mmax <= 8 ? 8 : mmax <= 16 ? 16 : mmax <= 32 ? 32 : 64;
  const int kg = kb < 16 ? 16 : kb;
  return cols < kg ? cols : kg;  // wider windows fall back to the separate passes
}

hipError_t launch_batch_init(BInst* inst, int count, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(p4::k_batch_init, dim3(count), dim3(kWG), 0, st, inst, count);
  return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned* counter, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(p4::k_batch_reset, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& b, int grid, int kbucket, bool gram, int stage_cols,
                        hipStream_t st, int pairs) {
  return pairs == 2 ? p2::launch_batch(b, grid, kbucket, gram, stage_cols, st)
                    : p4::launch_batch(b, grid, kbucket, gram, stage_cols, st);
}
#endif

}  // namespace aa
