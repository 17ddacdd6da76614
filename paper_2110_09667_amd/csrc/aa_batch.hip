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

#include "aa_passes.h"

namespace aa {

__device__ __forceinline__ Tail mk_tail(int op, int k) {
  Tail t{};
  t.op = op;
  t.k = k;
  return t;
}

template <int KB, bool GRAM>
struct BatchLds {
  static constexpr int KG = KB < 16 ? 16 : KB;          // Gram block bucket
  static constexpr int NACC = 2 * KB + 4;                // per-wave accumulators
  static constexpr int NPG = GRAM ? GramShape<KG>::NP : 1;
  static constexpr int NRED = NACC > NPG ? NACC : NPG;
  static constexpr int NSTAGE = GRAM ? GramShape<KG>::STAGE : 1;
  double acc[kWaves * NACC];
  double red[NRED];
  double c1[kMaxCols], c2[kMaxCols], cs[kMaxCols];
  double gc[KG], gs[KG];
  double sg[kMaxCols];
  int sslot[kMaxCols];
  union {                 // the Givens scratch is dead once the rotations exist
    double H[KB * KB];
    double stage[NSTAGE];
  };
};

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

// QRAdd (Alg. 2 with Algs. 3-6) of v as column k; k columns present.
template <int KB, class L>
__device__ void wg_qr_add(const BInst& I, int variant, unsigned flags, int k, const double* v,
                          L& lds) {
  const Small& sm = I.sm;
  double* slotk = I.Q + (int64_t)k * I.ld;
  double* Rcol = sm.R + (size_t)k * sm.cap;
  DotsArgs d{I.Q, I.ld, I.n, v, 0, nullptr, 0, 0};
  UpdArgs u{};
  u.Q = I.Q; u.ldq = I.ld; u.n = I.n; u.Qw = I.Q; u.dotcol = -1; u.dcgs2_p = -1;
  Tail tn = mk_tail(TAIL_NORM, k);
  tn.idx = 0;
  auto dots = [&](const DotsArgs& a, const Tail& t) {
    wg_pass(sm, t, a.nx + a.ny + (a.xx ? 1 : 0), lds,
            [&](double* acc) { dots_body(a, 0, 1, acc); });
  };
  auto update = [&](const UpdArgs& a, const Tail& t) {
    update_coefs(a, lds.c1, lds.c2, lds.cs);
    wg_pass(sm, t, (a.dotcol >= 0 ? 1 : 0) + (a.nrm ? 1 : 0), lds,
            [&](double* acc) { update_body(a, lds.c1, lds.c2, lds.cs, 0, 1, acc); });
  };
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
      dots(d, mk_tail(TAIL_CGS2_S, k));
      for (int j = threadIdx.x; j < KB; j += kWG) lds.cs[j] = (j < k) ? sm.coef0[j] : 0.0;
      Cgs2bArgs b{I.Q, I.ld, I.n, v, k, sm.coef0};
      wg_pass(sm, mk_tail(TAIL_CGS2_Z, k), k, lds,
              [&](double* acc) { cgs2b_stream_body(b, lds.cs, 0, 1, acc); });
      UpdArgs uc = u;
      uc.v = v; uc.out = slotk; uc.j0 = 0; uc.nc = k; uc.c1 = sm.coef0; uc.c2 = sm.coef1;
      uc.nrm = 1;
      update(uc, tn);
      break;
    }
    case AA_ICWY: {
      d.nx = k;
      d.y = I.Q + (int64_t)(k - 1) * I.ld;
      d.ny = k - 1;
      dots(d, mk_tail(TAIL_ICWY, k));
      UpdArgs ub = u;
      ub.v = v; ub.out = slotk; ub.j0 = 0; ub.nc = k; ub.c1 = sm.coef0; ub.nrm = 1;
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
      dots(d, ta);
      UpdArgs ub = u;
      ub.v = v; ub.out = slotk; ub.c1 = Rcol; ub.nrm = 1;
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

// QRDelete (Alg. 2): Givens rotations from R, one sweep over Q; ICWY also
// refreshes T (Gram of the rotated columns on the matrix cores).
template <int KB, bool GRAM, class L>
__device__ void wg_qr_delete(const BInst& I, int variant, int k, L& lds) {
  const Small& sm = I.sm;
  if (k <= 1) return;
  givens_body(sm, k, lds.H);
  __syncthreads();
  RotArgs r{I.Q, I.ld, I.n, k, sm.givens, 0};
  givens_coefs(r, sm.cap, lds.gc, lds.gs, L::KG);
  __syncthreads();
  if constexpr (GRAM) {
    if (variant == AA_ICWY) {
      constexpr int KG = L::KG;
      using S = GramShape<KG>;
      v4d acc[S::NBP];
      rotate_gram_body<KG>(r, lds.gc, lds.gs, 0, 1, lds.stage, acc);
      __syncthreads();
      gram_store<KG>(acc, lds.stage + (threadIdx.x >> 6) * S::NP);
      __syncthreads();
      const int kk = k - 1, nred = kk * (kk - 1) / 2;
      for (int c = threadIdx.x; c < nred; c += kWG) {
        double s = lds.stage[c];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += lds.stage[w * S::NP + c];
        lds.red[c] = s;
      }
      __syncthreads();
      run_tail(sm, mk_tail(TAIL_GRAM, kk), lds.red);
      __syncthreads();
      return;
    }
  }
  rotate_body(r, lds.gc, lds.gs, 0, 1);
  __syncthreads();
}

// One iteration of Alg. 1 for one instance (every thread of the workgroup).
// it, k: iteration index and column count on entry.  Returns the new state.
template <int KB, bool GRAM, class L>
__device__ BState wg_iteration(const BatchArgs& b, const BInst& I, BState st, L& lds) {
  const int tid = threadIdx.x;
  const Small& sm = I.sm;
  const double* x = b.ox ? b.ox : I.x;
  double* xn = b.oxn ? b.oxn : I.x;
  const double* g = b.og ? b.og : I.g;
  if (!b.og && I.dim > 0) {
    const double ih2 = 1.0 / (I.h * I.h);
    for (int64_t p = tid; p < I.n; p += kWG)
      I.g[p] = stencil_point(x, I.f, I.dim, I.s, ih2, I.omega, I.c, p);
    __syncthreads();
  }
  const int64_t it = st.iter;
  if (it == 0) {
    // Alg. 1 before the loop: x_1 = G(x_0), f_0 = G(x_0) - x_0
    HistArgs h{x, g, I.W, I.f_prev, I.g_prev, nullptr, xn, I.n, 1};
    wg_pass(sm, mk_tail(TAIL_FIRST, 0), 2, lds, [&](double* acc) { history_body(h, 0, 1, acc); });
    st.iter = 1;
    st.m_i = 0;
    st.res_norm = st.res0_norm = sqrt(sm.scal[S_RES]);
    return st;
  }
  const int m = I.m;
  const int m_i = (int)(it < m ? it : m);
  const int slot = (int)((it - 1) % m);
  HistArgs h{x, g, I.W, I.f_prev, I.g_prev, I.ring + (int64_t)slot * I.ld, nullptr, I.n, 0};
  wg_pass(sm, mk_tail(TAIL_RES, 0), 1, lds, [&](double* acc) { history_body(h, 0, 1, acc); });
  const double res = sqrt(sm.scal[S_RES]);
  st.res_norm = res;
  st.status = *sm.status;
  if (b.ov_iter < 0 && (res <= b.tol * st.res0_norm || it >= b.max_iter || st.status != AA_OK)) {
    st.active = 0;
    st.conv_iter = it;
    return st;
  }
  int k = st.k;
  if (it > m) {
    wg_qr_delete<KB, GRAM>(I, b.variant, k, lds);
    k -= 1;
  }
  wg_qr_add<KB>(I, b.variant, b.flags, k, I.W, lds);
  k += 1;
  DotsArgs d{I.Q, I.ld, I.n, I.f_prev, k, nullptr, 0, 0};
  wg_pass(sm, mk_tail(TAIL_RHS, k), k, lds, [&](double* acc) { dots_body(d, 0, 1, acc); });
  XupdArgs xa{I.ring, I.ld, m, (int)((it - m_i) % m), m_i, g, x, xn, I.n, sm.gamma};
  xupdate_coefs(xa, lds.sg, lds.sslot);
  wg_pass(sm, mk_tail(TAIL_STEP, 0), 1, lds,
          [&](double* acc) { xupdate_body(xa, lds.sg, lds.sslot, 0, 1, acc); });
  st.iter = it + 1;
  st.k = k;
  st.m_i = m_i;
  st.status = *sm.status;
  return st;
}

template <int KB, bool GRAM>
__global__ __launch_bounds__(kWG) void k_batch(BatchArgs b) {
  using L = BatchLds<KB, GRAM>;
  __shared__ L lds;
  __shared__ int s_idx;
  if (b.ov_iter >= 0) {  // fused single-instance step: host-held counters
    BState st = b.state[0];
    st.iter = b.ov_iter;
    st.k = b.ov_k;
    st.active = 1;
    const BState out = wg_iteration<KB, GRAM>(b, b.inst[0], st, lds);
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
    const BState st = b.state[j];
    if (!st.active) continue;
    const BState out = wg_iteration<KB, GRAM>(b, b.inst[j], st, lds);
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
static hipError_t launch_kb(const BatchArgs& b, int grid, int kb, hipStream_t st) {
  switch (kb) {
    case 8: hipLaunchKernelGGL((k_batch<8, GRAM>), dim3(grid), dim3(kWG), 0, st, b); break;
    case 16: hipLaunchKernelGGL((k_batch<16, GRAM>), dim3(grid), dim3(kWG), 0, st, b); break;
    case 32: hipLaunchKernelGGL((k_batch<32, GRAM>), dim3(grid), dim3(kWG), 0, st, b); break;
    case 64: hipLaunchKernelGGL((k_batch<64, GRAM>), dim3(grid), dim3(kWG), 0, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& b, int grid, int kbucket, bool gram, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  return gram ? launch_kb<true>(b, grid, kbucket, st) : launch_kb<false>(b, grid, kbucket, st);
}

hipError_t launch_batch_init(BInst* inst, int count, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_batch_init, dim3(count), dim3(kWG), 0, st, inst, count);
  return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned* counter, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

}  // namespace aa
