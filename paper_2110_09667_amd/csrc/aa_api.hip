// aa_api.hip -- host side of the C ABI declared in include/aa.h.
//
// The context tracks the iteration index and the column count k on the host
// (both evolve deterministically), carves the caller's workspace into Q, the
// history of G differences, the work vectors and the small dense block, and
// enqueues the kernel sequence of each step on the context's stream.
#include <stdlib.h>
#include <string.h>

#include <limits.h>
#include <new>
#include <vector>

#include "aa_internal.h"

using namespace aa;

struct aa_ctx {
  int64_t n = 0, ldq = 0;
  int m = 0, cap = 0, variant = 0;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  double* Q = nullptr;      // ldq x cap
  double* ring = nullptr;   // ldq x m (Delta g history), AA only
  double* W = nullptr;      // ldq (Delta f / MGS work vector)
  double* f_prev = nullptr; // ldq, AA only
  double* g_prev = nullptr; // ldq, AA only
  Small sm{};
  // workgroups of the streaming passes: two per compute unit (measured at n =
  // 2^26 and the 256^3 step against 768 and 1024: 1-2 % faster; with four per
  // CU the update pass runs at 5.47 TB/s, with two at 5.62)
  int grid_stream_max = 512;
  int grid_gram_max = 1024;    // workgroups of the ICWY Gram pass
  int64_t iter = 0;
  int k = 0, m_i = 0;
  int64_t syncs_add = 0, syncs_del = 0, syncs_rhs = 0;
  // stopping rule (aa_set_stop) and its device state
  StopState* stop_dev = nullptr;
  int stop_mode = kStopNone;
  double stop_tol = 0.0;
  int64_t max_iter = 0;  // 0: no cap
  // fused single-workgroup step for small n (aa_batch.hip)
  BInst* d_binst = nullptr;
  BState* d_bstate = nullptr;
  int64_t fused_max = 0;  // set by aa_init: kFusedWork / m
  bool one_wg_ok = true;  // the variant and flags have a one-workgroup step
  // steady-state iterations replayed as HIP graphs (aa_set_graph): one per
  // ring-slot phase (i - 1) mod m, valid for the caller pointers it captured
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    const double* x = nullptr;
    const double* g = nullptr;
    double* xn = nullptr;
    int64_t d_add = 0, d_del = 0, d_rhs = 0;
  };
  bool graph_on = false;
  std::vector<StepGraph> graphs;
  // per-launch timing (aa_profile_enable)
  bool prof_on = false;
  std::vector<hipEvent_t> ev;   // per launch p: 3p start, 3p+1 pass end, 3p+2 stop
  std::vector<int> ev_kind;
  std::vector<char> ev_mid;
  int ev_used = 0;
  double prof_ms[AA_K_COUNT] = {};
  int64_t prof_launches[AA_K_COUNT] = {};
  double prof_bytes[AA_K_COUNT] = {};
};

namespace {

constexpr size_t kAlign = 256;
// Reduction partials: room for kMaxRed values from 4096 workgroups (the
// largest streaming grid), which also covers the Gram pass below.
constexpr size_t kPartials = (size_t)kMaxRed * 8192;  // 12.8 MB: the 63-column Gram at 512 workgroups

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t leading_dim(int64_t n) {
  // The column stride decides how the columns of one row tile fall on the HBM
  // channels.  Measured at n = 2^26 with eight column streams read at once:
  // 7.0 TB/s at a stride of n + 1024 doubles (columns 8 KiB apart modulo the
  // interleave), 6.3 TB/s at n + 64 and 6.0-6.2 TB/s at n + 2048 or n + 4096.
  // Long columns therefore get a stride of 1024 (mod 2048) doubles; short
  // ones are padded to 64 doubles, off powers of two.
  int64_t ld = (n + 63) / 64 * 64;
  if (ld >= 65536) return (ld + 2047) / 2048 * 2048 + 1024;
  if (ld >= 4096 && (ld & (ld - 1)) == 0) ld += 64;
  else if (ld % 4096 == 0) ld += 64;
  return ld;
}

struct Layout {
  int64_t ldq;
  size_t off_Q, off_ring, off_W, off_fp, off_gp, off_R, off_T, off_c0, off_c1, off_gam,
      off_giv, off_scal, off_status, off_stop, off_part, off_binst, off_bstate, total;
};

Layout make_layout(int64_t n, int m, unsigned flags) {
  Layout L{};
  const int cap = m;
  L.ldq = leading_dim(n);
  const size_t vec = (size_t)L.ldq * sizeof(double);
  size_t o = 0;
  L.off_Q = o; o = align_up(o + vec * cap);
  if (!(flags & AA_QR_ONLY)) {
    L.off_ring = o; o = align_up(o + vec * m);
    L.off_fp = o; o = align_up(o + vec);
    L.off_gp = o; o = align_up(o + vec);
  }
  L.off_W = o; o = align_up(o + vec);
  L.off_R = o; o = align_up(o + sizeof(double) * cap * cap);
  L.off_T = o; o = align_up(o + sizeof(double) * cap * cap);
  L.off_c0 = o; o = align_up(o + sizeof(double) * cap);
  L.off_c1 = o; o = align_up(o + sizeof(double) * cap);
  L.off_gam = o; o = align_up(o + sizeof(double) * cap);
  L.off_giv = o; o = align_up(o + sizeof(double) * 2 * cap);
  L.off_scal = o; o = align_up(o + sizeof(double) * S_COUNT);
  L.off_status = o; o = align_up(o + sizeof(int));
  L.off_stop = o; o = align_up(o + sizeof(StopState));
  const size_t part = kPartials;
  L.off_part = o; o = align_up(o + sizeof(double) * part);
  L.off_binst = o; o = align_up(o + sizeof(BInst));
  L.off_bstate = o; o = align_up(o + sizeof(BState));
  L.total = o;
  return L;
}

bool valid_variant(int v) { return v >= AA_MGS && v <= AA_DCGS2_LAG; }

// Variants whose first QRAdd pass the fused delete can take over.
bool fuse_delete_ok(int v) { return v == AA_CGS2 || v == AA_DCGS2 || v == AA_ICWY; }

aa_status hip_ok(hipError_t e) { return e == hipSuccess ? AA_OK : AA_EHIP; }

int grid_for(const aa_ctx* c, int64_t rows_per_wg, int gmax) {
  int64_t g = (c->n + rows_per_wg - 1) / rows_per_wg;
  if (g > gmax) g = gmax;
  if (g < 1) g = 1;
  return (int)g;
}

int grid_stream(const aa_ctx* c) { return grid_for(c, kTile, c->grid_stream_max); }
int grid_rows(const aa_ctx* c, int gmax) { return grid_for(c, kWG, gmax); }

constexpr int kEventPairs = 4096;

// Default reach of the one-workgroup step: n * m <= kFusedWork.  One
// workgroup streams ~23 GB/s, so its iteration costs ~2 ns per n*m element on
// top of ~45 us; the grid-wide passes cost ~90 us at small n (about a dozen
// dependent launches).  They break even near n * m = 20480 (measured on the
// 3D workload: n = 13824, m = 20 took 0.65 ms in one workgroup; n = 32768
// took 0.09 ms on the grid path).
constexpr int64_t kFusedWork = 20480;

hipError_t prof_drain(aa_ctx* c) {
  if (c->ev_used == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(c->ev[3 * (c->ev_used - 1) + 2]);
  if (e != hipSuccess) return e;
  for (int p = 0; p < c->ev_used; ++p) {
    float ms = 0.f;
    if (c->ev_mid[p]) {
      e = hipEventElapsedTime(&ms, c->ev[3 * p], c->ev[3 * p + 1]);
      if (e != hipSuccess) return e;
      c->prof_ms[c->ev_kind[p]] += ms;
      e = hipEventElapsedTime(&ms, c->ev[3 * p + 1], c->ev[3 * p + 2]);
      if (e != hipSuccess) return e;
      c->prof_ms[AA_K_FINALIZE] += ms;
    } else {
      e = hipEventElapsedTime(&ms, c->ev[3 * p], c->ev[3 * p + 2]);
      if (e != hipSuccess) return e;
      c->prof_ms[c->ev_kind[p]] += ms;
    }
  }
  c->ev_used = 0;
  return hipSuccess;
}

// Enqueue one pass; with profiling on, bracket it with events (plus one
// between the pass kernel and its finalize kernel, if it has one) and account
// `vecs` algorithmic vector transfers (8 n bytes each) to its kind.
template <class F>
hipError_t timed(aa_ctx* c, int kind, double vecs, F&& launch) {
  if (!c->prof_on) return launch();
  if (c->ev_used == kEventPairs) {
    hipError_t e = prof_drain(c);
    if (e != hipSuccess) return e;
  }
  const int p = c->ev_used;
  hipError_t e = hipEventRecord(c->ev[3 * p], c->stream);
  if (e != hipSuccess) return e;
  set_profile_mid(c->ev[3 * p + 1]);
  e = launch();
  const bool mid = profile_mid_used();
  set_profile_mid(nullptr);
  if (e != hipSuccess) return e;
  e = hipEventRecord(c->ev[3 * p + 2], c->stream);
  if (e != hipSuccess) return e;
  c->ev_kind[p] = kind;
  c->ev_mid[p] = mid ? 1 : 0;
  c->ev_used = p + 1;
  c->prof_launches[kind] += 1;
  c->prof_bytes[kind] += vecs * 8.0 * (double)c->n;
  if (mid) c->prof_launches[AA_K_FINALIZE] += 1;
  return hipSuccess;
}

Tail tail(int op, int k) {
  Tail t{};
  t.op = op;
  t.k = k;
  return t;
}

// QRAdd of d_v as column k (Algs. 3-6); d_v is read-only.  With f non-null
// (AA_FUSE_RHS, k >= 1, not MGS) the passes also form c = Q^T f of the grown
// basis and the last pass's tail solves R gamma = c (Alg. 2, last line):
// the first pass adds Q^T f to its block dot products, the norm pass adds
// w^T f (c_k = w^T f / R_kk); *rhs_done reports whether that happened.
aa_status qr_add_impl(aa_ctx* c, const double* v, const double* f = nullptr,
                      bool* rhs_done = nullptr, bool first_done = false) {
  const int k = c->k;
  if (k >= c->cap) return AA_ESTATE;
  if (first_done && (k == 0 || c->variant == AA_MGS)) return AA_EINVAL;
  const bool fuse = f != nullptr && k >= 1 && k + 1 <= 64 && c->variant != AA_MGS;
  if (rhs_done) *rhs_done = fuse;
  const int zf = fuse ? 1 : 0;  // one more vector read by each fused pass
  const hipStream_t st = c->stream;
  const int G = grid_stream(c);
  double* slotk = c->Q + (int64_t)k * c->ldq;
  double* Rcol = c->sm.R + (size_t)k * c->sm.cap;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };

  DotsArgs d{c->Q, c->ldq, c->n, v, 0, nullptr, 0, 0};
  UpdArgs u{};
  u.Q = c->Q; u.ldq = c->ldq; u.n = c->n; u.Qw = c->Q; u.dotcol = -1; u.dcgs2_p = -1;
  Tail tn = tail(TAIL_NORM, k);
  tn.idx = 0;

  if (k == 0) {
    // Alg. 2 with i = 1 (and every QRAdd into an empty window): normalize.
    d.xx = 1;
    chk(timed(c, AA_K_DOTS, 1, [&] { return launch_dots(d, c->sm, tn, G, st); }));
    c->syncs_add += 1;
  } else {
    switch (c->variant) {
      case AA_MGS: {
        Tail t0 = tail(TAIL_MGS_R, k);
        t0.row = 0;
        d.nx = 1;
        chk(timed(c, AA_K_DOTS, 2, [&] { return launch_dots(d, c->sm, t0, G, st); }));
        const double* cur = v;
        for (int j = 1; j < k; ++j) {
          UpdArgs uj = u;
          uj.v = cur; uj.out = c->W; uj.j0 = j - 1; uj.nc = 1; uj.c1 = Rcol; uj.dotcol = j;
          uj.rev = (j & 1);  // alternate with the previous pass (dots: forward)
          Tail tj = tail(TAIL_MGS_R, k);
          tj.row = j;
          chk(timed(c, AA_K_UPDATE, 4, [&] { return launch_update(uj, c->sm, tj, G, st); }));
          cur = c->W;
        }
        UpdArgs uk = u;
        uk.v = cur; uk.out = slotk; uk.j0 = k - 1; uk.nc = 1; uk.c1 = Rcol; uk.nrm = 1;
        uk.rev = (k & 1);
        chk(timed(c, AA_K_UPDATE, 3, [&] { return launch_update(uk, c->sm, tn, G, st); }));
        c->syncs_add += k + 1;
        break;
      }
      case AA_CGS2: {
        d.nx = k;
        Tail ts = tail(TAIL_CGS2_S, k);
        if (fuse) {
          d.z = f; d.nz = k;
          ts.rhs = 1; ts.zoff = k;
        }
        if (!first_done)
          chk(timed(c, AA_K_DOTS, k + 1 + zf,
                    [&] { return launch_dots(d, c->sm, ts, G, st); }));
        // the three passes alternate direction: dots forward, this pass
        // backward, the update forward
        Cgs2bArgs b{c->Q, c->ldq, c->n, v, k, c->sm.coef0, 1};
        const int Gb = grid_rows(c, c->grid_stream_max);
        chk(timed(c, AA_K_CGS2B, k + 1,
                  [&] { return launch_cgs2b(b, c->sm, tail(TAIL_CGS2_Z, k), Gb, st); }));
        UpdArgs uc = u;
        uc.v = v; uc.out = slotk; uc.j0 = 0; uc.nc = k; uc.c1 = c->sm.coef0; uc.c2 = c->sm.coef1;
        uc.nrm = 1;
        uc.rev = 0;  // after the backward second pass
        if (fuse) {
          uc.rhsv = f;
          tn.rhs = 1;
        }
        chk(timed(c, AA_K_UPDATE, k + 2 + zf, [&] { return launch_update(uc, c->sm, tn, G, st); }));
        c->syncs_add += first_done ? 2 : 3;
        break;
      }
      case AA_ICWY: {
        d.nx = k;
        d.y = c->Q + (int64_t)(k - 1) * c->ldq;
        d.ny = k - 1;
        Tail ti = tail(TAIL_ICWY, k);
        if (fuse) {
          d.z = f; d.nz = k;
          ti.rhs = 1; ti.zoff = 2 * k - 1;
        }
        if (!first_done)
          chk(timed(c, AA_K_DOTS, k + 1 + zf,
                    [&] { return launch_dots(d, c->sm, ti, G, st); }));
        UpdArgs ub = u;
        ub.v = v; ub.out = slotk; ub.j0 = 0; ub.nc = k; ub.c1 = c->sm.coef0; ub.nrm = 1;
        ub.rev = 1;  // after a forward pass over the same columns
        if (fuse) {
          ub.rhsv = f;
          tn.rhs = 1;
        }
        chk(timed(c, AA_K_UPDATE, k + 2 + zf, [&] { return launch_update(ub, c->sm, tn, G, st); }));
        c->syncs_add += first_done ? 1 : 2;
        break;
      }
      case AA_DCGS2: {
        const int m_i = k + 1;
        const bool reorth = (c->flags & AA_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
        d.nx = k;
        d.y = c->Q + (int64_t)(k - 1) * c->ldq;
        d.ny = reorth ? k - 1 : 0;
        Tail ta = tail(TAIL_DCGS2, k);
        ta.reorth = reorth;
        ta.literal = (c->flags & AA_DCGS2_LITERAL) ? 1 : 0;
        if (fuse) {
          d.z = f; d.nz = k;
          ta.rhs = 1; ta.zoff = k + d.ny;
        }
        if (!first_done)
          chk(timed(c, AA_K_DOTS, k + 1 + zf, [&] { return launch_dots(d, c->sm, ta, G, st); }));
        UpdArgs ub = u;
        ub.v = v; ub.out = slotk; ub.c1 = Rcol; ub.nrm = 1;
        ub.rev = 1;  // after a forward pass over the same columns
        if (fuse) {
          ub.rhsv = f;
          tn.rhs = 1;
        }
        if (reorth) {
          ub.dcgs2_p = k - 1; ub.reorth = 1; ub.s = c->sm.coef1; ub.j0 = 0; ub.nc = k - 1;
        } else {
          ub.j0 = 0; ub.nc = k;
        }
        chk(timed(c, AA_K_UPDATE, k + (reorth ? 3 : 2) + zf,
                  [&] { return launch_update(ub, c->sm, tn, G, st); }));
        c->syncs_add += first_done ? 1 : 2;
        break;
      }
      case AA_DCGS2_LAG: {
        // DCGS-2 with the normalization lagged (Sec. 3.4): one reduction
        // [Q^T v | Q^T q_{k-1} | v^T v (| Q^T f, v^T f)] finishes the previous
        // column and projects v; the update pass writes both columns already
        // normalized (no reduction, no scale pass).
        const int p = k - 1;
        d.nx = k;
        d.y = c->Q + (int64_t)p * c->ldq;
        d.ny = k;
        d.xx = 1;
        Tail tl = tail(TAIL_DCGS2_LAG, k);
        tl.idx = 2 * k;
        if (fuse) {
          d.z = f; d.nz = k; d.xz = 1;
          tl.rhs = 1; tl.zoff = 2 * k; tl.idx = 3 * k;
        }
        chk(timed(c, AA_K_DOTS, k + 1 + zf, [&] { return launch_dots(d, c->sm, tl, G, st); }));
        UpdArgs ub = u;
        ub.v = v; ub.out = slotk; ub.c1 = c->sm.coef0; ub.s = c->sm.coef1;
        ub.dcgs2_p = p; ub.reorth = 1; ub.j0 = 0; ub.nc = p;
        ub.pdiv = c->sm.scal + S_RHO; ub.odiv = c->sm.scal + S_RKK;
        ub.rev = 1;  // after a forward pass over the same columns
        chk(timed(c, AA_K_UPDATE, k + 3, [&] { return launch_update(ub, c->sm, tail(TAIL_NONE, k), G, st); }));
        c->syncs_add += 1;
        if (e != hipSuccess) return AA_EHIP;
        c->k = k + 1;
        return AA_OK;
      }
      default:
        return AA_EINVAL;
    }
  }
  ScaleArgs sa{k == 0 ? v : slotk, slotk, c->n, c->sm.R, k, c->sm.cap, c->sm.stop, c->sm.status};
  chk(timed(c, AA_K_SCALE, 2, [&] { return launch_scale(sa, c->sm, st); }));
  if (e != hipSuccess) return AA_EHIP;
  c->k = k + 1;
  return AA_OK;
}

// refresh_next: a QRAdd follows (inside aa_step), which recomputes the last
// row of ICWY's T from its first reduction before anything reads it, so the
// Gram leaves the last rotated column out (at m = 50: 48 columns, 6 MFMA block
// pairs per 4 rows instead of 10).  The standalone QRDelete refreshes all of T.
aa_status qr_delete_impl(aa_ctx* c, bool refresh_next) {
  const int k = c->k;
  if (k <= 0) return AA_ESTATE;
  if (k == 1) {
    c->k = 0;
    return AA_OK;
  }
  // ICWY with AA_ICWY_T_TRANSFORM: T follows the rotations in the Givens
  // kernel (no reduction); otherwise the rotation pass refreshes it.
  const bool transform = c->variant == AA_ICWY && (c->flags & AA_ICWY_T_TRANSFORM);
  hipError_t e = timed(c, AA_K_GIVENS, 0,
                       [&] { return launch_givens(c->sm, k, c->stream, transform); });
  if (e != hipSuccess) return AA_EHIP;
  const bool gram = c->variant == AA_ICWY && !transform;
  const int drop = gram && refresh_next ? 1 : 0;
  RotArgs r{c->Q, c->ldq, c->n, k, c->sm.givens, gram ? 1 : 0, nullptr, nullptr, 0, drop};
  const int ng = gram_cols(r);  // columns of the Gram
  int gmax = c->grid_stream_max;
  if (gram) {  // ng(ng-1)/2 pair sums per workgroup must fit the partials
    const int64_t pairs = (int64_t)ng * (ng - 1) / 2;
    const int64_t cap = pairs > 0 ? (int64_t)kPartials / pairs : c->grid_gram_max;
    gmax = (int)(c->grid_gram_max < cap ? c->grid_gram_max : cap);
  }
  const int G = grid_rows(c, gmax);
  e = timed(c, AA_K_ROTATE, 2 * k - 1,
            [&] { return launch_rotate(r, c->sm, tail(TAIL_GRAM, ng), G, c->stream); });
  if (e != hipSuccess) return AA_EHIP;
  if (gram) c->syncs_del += 1;
  c->k = k - 1;
  return AA_OK;
}

// The tail of the QRAdd's first pass (block dot products) for the variant
// with k columns present, as qr_add_impl builds it, and where its inputs sit
// in that pass's reduced values: Q^T v at 0, the Gram row of q_{k-1}
// (ICWY; DCGS-2 when it reorthogonalizes) at k, Q^T f after them.
Tail first_pass_tail(const aa_ctx* c, int k, bool rhs) {
  Tail t{};
  t.k = k;
  switch (c->variant) {
    case AA_CGS2:
      t.op = TAIL_CGS2_S;
      t.zoff = k;
      break;
    case AA_ICWY:
      t.op = TAIL_ICWY;
      t.zoff = 2 * k - 1;
      break;
    default: {  // DCGS-2
      const int m_i = k + 1;
      t.op = TAIL_DCGS2;
      t.reorth = (c->flags & AA_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
      t.literal = (c->flags & AA_DCGS2_LITERAL) ? 1 : 0;
      t.zoff = k + (t.reorth ? k - 1 : 0);
    }
  }
  t.rhs = rhs ? 1 : 0;
  return t;
}

// A full window with CGS-2, DCGS-2 or ICWY (AA_FUSE_DELETE): QRDelete's
// rotation pass also stages v (and f) beside the rotated columns, and the
// Gram of [Q v f] on the matrix cores yields at once ICWY's T refresh and
// every block dot product the QRAdd's first pass would compute (Q^T v, the
// Gram row of the last column, Q^T f).  The finalize rearranges them into
// that pass's layout and runs its tail; qr_add_impl then continues from the
// second pass.  One pass over Q and one reduction fewer per iteration.
aa_status fused_delete_add(aa_ctx* c, const double* v, const double* f, bool* rhs_done) {
  const int k = c->k, kk = k - 1;
  const int naug = f ? 2 : 1;
  const hipStream_t st = c->stream;
  hipError_t e = timed(c, AA_K_GIVENS, 0, [&] { return launch_givens(c->sm, k, st); });
  if (e != hipSuccess) return AA_EHIP;
  RotArgs r{c->Q, c->ldq, c->n, k, c->sm.givens, 1, v, f, naug};
  const int na = kk + naug;
  const int64_t pairs = (int64_t)na * (na - 1) / 2;
  const int64_t cap = pairs > 0 ? (int64_t)kPartials / pairs : c->grid_gram_max;
  const int gmax = (int)(c->grid_gram_max < cap ? c->grid_gram_max : cap);
  Tail tg = first_pass_tail(c, kk, f != nullptr);
  tg.inner = tg.op;
  tg.op = TAIL_GRAM_ADD;
  tg.gram_t = c->variant == AA_ICWY ? 1 : 0;
  e = timed(c, AA_K_ROTATE, 2 * k - 1 + naug,
            [&] { return launch_rotate(r, c->sm, tg, grid_rows(c, gmax), st); });
  if (e != hipSuccess) return AA_EHIP;
  c->syncs_del += 1;
  c->k = kk;
  return qr_add_impl(c, v, f, rhs_done, true);
}

aa_status rhs_impl(aa_ctx* c, const double* f) {
  DotsArgs d{c->Q, c->ldq, c->n, f, c->k, nullptr, 0, 0};
  const int G = grid_stream(c);
  hipError_t e = timed(c, AA_K_DOTS, c->k + 1,
                       [&] { return launch_dots(d, c->sm, tail(TAIL_RHS, c->k), G, c->stream); });
  c->syncs_rhs += 1;
  return hip_ok(e);
}

// Algorithmic vectors moved by QRAdd with k columns present (Algs. 3-6).
double add_vectors(int variant, unsigned flags, int k) {
  if (k == 0) return 3;
  switch (variant) {
    case AA_MGS: return 4.0 * k + 3;
    case AA_CGS2: return 3.0 * k + 6;
    case AA_ICWY: return 2.0 * k + 5;
    case AA_DCGS2_LAG: return 2.0 * k + 4;
    default: {
      const int m_i = k + 1;
      const bool reorth = (flags & AA_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
      return 2.0 * k + (reorth ? 6 : 5);
    }
  }
}

int64_t add_syncs(int variant, int k) {
  if (k == 0) return 1;
  switch (variant) {
    case AA_MGS: return k + 1;
    case AA_CGS2: return 3;
    case AA_DCGS2_LAG: return 1;
    default: return 2;
  }
}

// One iteration in a single workgroup (the batched step with one instance and
// the host's counters); same sequence and arithmetic as the grid path.
aa_status fused_step(aa_ctx* c, const double* x, const double* g, double* x_next) {
  BatchArgs a{};
  a.inst = c->d_binst;
  a.state = c->d_bstate;
  a.count = 1;
  a.variant = c->variant;
  a.flags = c->flags;
  a.tol = 0.0;
  a.max_iter = INT64_MAX;
  a.ox = x; a.og = g; a.oxn = x_next;
  a.ov_iter = c->iter;
  a.ov_k = c->k;
  a.stop_mode = c->stop_mode;
  a.stop_tol = c->stop_tol;
  const int kb = c->m <= 8 ? 8 : c->m <= 16 ? 16 : c->m <= 32 ? 32 : 64;
  const bool gram = batch_needs_gram(c->variant, c->flags);
  // model bytes and reduction counts of this iteration
  double vecs = 5;
  const int64_t i = c->iter;
  int k = c->k;
  if (i > 0) {
    // the same decisions as the one-workgroup kernel (aa_batch.hip wg_front)
    const int m_i = (int)(i < c->m ? i : c->m);
    const bool fold = (c->flags & AA_FUSE_RHS) && c->variant != AA_MGS && c->m + 1 <= 64;
    const int kg = kb < 16 ? 16 : kb;
    bool del_fused = false;
    vecs = 8;
    if (i > c->m) {
      del_fused = (c->flags & AA_FUSE_DELETE) && c->variant != AA_MGS && k >= 2 &&
                  k - 1 + (fold ? 2 : 1) <= kg;
      vecs += 2.0 * k - 1 + (del_fused ? (fold ? 2 : 1) : 0);
      if ((c->variant == AA_ICWY && k > 1) || del_fused) c->syncs_del += 1;
      k -= 1;
    }
    double add = add_vectors(c->variant, c->flags, k);
    int64_t asy = add_syncs(c->variant, k);
    if (del_fused) {  // the first pass's block dot products came with the rotation
      add -= k + 1;
      asy -= 1;
    }
    const bool rhs_folded = fold && k >= 1;
    if (rhs_folded) add += del_fused ? 1 : 2;  // f in the first (unless fused) and norm passes
    vecs += add;
    c->syncs_add += asy;
    if (!rhs_folded) {
      vecs += k + 2;  // Q^T f_i over the k + 1 columns after the add
      c->syncs_rhs += 1;
    }
    vecs += m_i + 3;
  }
  hipError_t e = timed(c, AA_K_FUSED, vecs,
                       [&] { return launch_batch(a, 1, kb, gram, batch_stage_cols(c->m, c->variant, c->flags),
                                           c->stream); });
  if (e != hipSuccess) return AA_EHIP;
  if (i == 0) {
    c->iter = 1;
    c->m_i = 0;
  } else {
    c->m_i = (int)(i < c->m ? i : c->m);
    c->k = k + 1;
    c->iter = i + 1;
  }
  return AA_OK;
}

void drop_graphs(aa_ctx* c) {
  for (auto& sg : c->graphs)
    if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
  c->graphs.clear();
}

}  // namespace

namespace aa {

aa_ctx* view_create(const BInst& I, int variant, unsigned flags, double* partials,
                    StopState* stop, int64_t iter, int k, int m_i, double tol, int64_t max_iter,
                    hipStream_t st) {
  aa_ctx* c = new (std::nothrow) aa_ctx();
  if (!c) return nullptr;
  c->n = I.n;
  c->ldq = I.ld;
  c->m = I.m;
  c->cap = I.m;
  c->variant = variant;
  c->flags = flags & ~(unsigned)AA_BATCH_LEARNED;
  c->stream = st;
  c->Q = I.Q;
  c->ring = I.ring;
  c->W = I.W;
  c->f_prev = I.f_prev;
  c->g_prev = I.g_prev;
  c->sm = I.sm;
  c->sm.partials = partials;
  c->sm.npart = 0;  // the split path's buffer: sums in the finalize
  c->sm.stop = nullptr;
  c->stop_dev = stop;
  c->one_wg_ok = false;
  c->fused_max = 0;
  c->iter = iter;
  c->k = k;
  c->m_i = m_i;
  c->stop_mode = tol > 0.0 ? kStopResidual : kStopNone;
  c->stop_tol = tol > 0.0 ? tol : 0.0;
  // the batch stops at the start of iteration max_iter; aa_step's cap lets
  // iterations up to c->max_iter run
  c->max_iter = max_iter > 1 ? max_iter - 1 : 1;
  return c;
}

void view_counters(const aa_ctx* c, int64_t* iter, int* k, int* m_i) {
  *iter = c->iter;
  *k = c->k;
  *m_i = c->m_i;
}

void view_destroy(aa_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  delete c;
}

}  // namespace aa

extern "C" {

aa_status aa_workspace_size(int64_t n, int m, int variant, unsigned flags, size_t* bytes) {
  if (!bytes || n < 1 || m < 1 || m > AA_MAX_COLS || !valid_variant(variant)) return AA_EINVAL;
  if (variant == AA_ICWY && m > 64) return AA_EINVAL;
  // The least-squares solve (one wave, one lane per row of R) reaches 64
  // columns: the 65th column exists only for the QR update on its own.
  if (m > 64 && !(flags & AA_QR_ONLY)) return AA_EINVAL;
  *bytes = make_layout(n, m, flags).total;
  return AA_OK;
}

aa_status aa_init(aa_ctx** ctx, int64_t n, int m, int variant, unsigned flags,
                  void* d_workspace, size_t bytes, void* stream) {
  if (!ctx) return AA_EINVAL;
  *ctx = nullptr;
  size_t need = 0;
  aa_status s = aa_workspace_size(n, m, variant, flags, &need);
  if (s != AA_OK) return s;
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0) return AA_EINVAL;
  if (bytes < need) return AA_ENOSPACE;
  aa_ctx* c = new (std::nothrow) aa_ctx();
  if (!c) return AA_EINVAL;
  const Layout L = make_layout(n, m, flags);
  char* base = (char*)d_workspace;
  c->n = n;
  c->ldq = L.ldq;
  c->m = m;
  // the one-workgroup step implements Algs. 3-6 with the paper's T refresh
  c->one_wg_ok = variant != AA_DCGS2_LAG && !(flags & AA_ICWY_T_TRANSFORM);
  c->fused_max = c->one_wg_ok ? kFusedWork / m : 0;
  c->cap = m;
  c->variant = variant;
  c->flags = flags;
  c->stream = (hipStream_t)stream;
  c->Q = (double*)(base + L.off_Q);
  if (!(flags & AA_QR_ONLY)) {
    c->ring = (double*)(base + L.off_ring);
    c->f_prev = (double*)(base + L.off_fp);
    c->g_prev = (double*)(base + L.off_gp);
  }
  c->W = (double*)(base + L.off_W);
  c->sm.R = (double*)(base + L.off_R);
  c->sm.T = (double*)(base + L.off_T);
  c->sm.coef0 = (double*)(base + L.off_c0);
  c->sm.coef1 = (double*)(base + L.off_c1);
  c->sm.gamma = (double*)(base + L.off_gam);
  c->sm.givens = (double*)(base + L.off_giv);
  c->sm.scal = (double*)(base + L.off_scal);
  c->sm.status = (int*)(base + L.off_status);
  c->sm.partials = (double*)(base + L.off_part);
  c->sm.npart = (int64_t)kPartials;
  c->sm.cap = m;
  c->sm.stop = nullptr;  // set only while an AA step is enqueued
  c->stop_dev = (StopState*)(base + L.off_stop);
  Small s0 = c->sm;
  s0.stop = c->stop_dev;
  if (launch_init_small(s0, c->stream) != hipSuccess) {
    delete c;
    return AA_EHIP;
  }
  if (!(flags & AA_QR_ONLY) && m <= 64) {
    // descriptor of this context for the fused single-workgroup step
    BInst I{};
    I.n = n; I.ld = c->ldq; I.m = m; I.dim = 0;
    I.f_prev = c->f_prev; I.g_prev = c->g_prev; I.W = c->W; I.Q = c->Q; I.ring = c->ring;
    I.sm = c->sm;
    I.sm.stop = c->stop_dev;  // the one-workgroup step is an AA step
    BState st{};
    st.conv_iter = -1;
    st.active = 1;
    c->d_binst = (BInst*)(base + L.off_binst);
    c->d_bstate = (BState*)(base + L.off_bstate);
    if (hipMemcpyAsync(c->d_binst, &I, sizeof(I), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_bstate, &st, sizeof(st), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      delete c;
      return AA_EHIP;
    }
  }
  *ctx = c;
  return AA_OK;
}

aa_status aa_set_stream(aa_ctx* c, void* stream) {
  if (c) drop_graphs(c);
  if (!c) return AA_EINVAL;
  c->stream = (hipStream_t)stream;
  return AA_OK;
}


// While an AA step is enqueued its launches carry the device stop state.
struct StepScope {
  aa_ctx* c;
  explicit StepScope(aa_ctx* cc) : c(cc) { c->sm.stop = c->stop_dev; }
  ~StepScope() { c->sm.stop = nullptr; }
};

// One iteration of Alg. 1 enqueued kernel by kernel (host sequencing).
static aa_status step_enqueue(aa_ctx* c, const double* x, const double* g,
                              double* x_next) {
  if (c->d_binst && c->n <= c->fused_max) return fused_step(c, x, g, x_next);
  StepScope scope(c);
  const hipStream_t st = c->stream;
  const int G = grid_stream(c);
  if (c->iter == 0) {
    // Alg. 1 before the loop: x_1 = G(x_0), f_0 = G(x_0) - x_0.
    HistArgs h{x, g, c->W, c->f_prev, c->g_prev, nullptr, x_next, c->n, 1};
    if (timed(c, AA_K_HISTORY, 5,
              [&] { return launch_history(h, c->sm, tail(TAIL_FIRST, 0), G, st); }) != hipSuccess)
      return AA_EHIP;
    c->iter = 1;
    c->m_i = 0;
    return AA_OK;
  }
  const int64_t i = c->iter;
  const int m = c->m;
  const int m_i = (int)(i < m ? i : m);
  const int slot = (int)((i - 1) % m);
  HistArgs h{x, g, c->W, c->f_prev, c->g_prev, c->ring + (int64_t)slot * c->ldq, nullptr,
             c->n, 0};
  Tail tr = tail(TAIL_RES, c->k);  // the stopping test at the start of iteration i
  tr.stop_mode = c->stop_mode;
  tr.stop_tol = c->stop_tol;
  tr.m_i = c->m_i;
  if (timed(c, AA_K_HISTORY, 8,
            [&] { return launch_history(h, c->sm, tr, G, st); }) != hipSuccess)
    return AA_EHIP;
  aa_status s = AA_OK;
  bool rhs_done = false;
  const bool fuse_rhs = (c->flags & AA_FUSE_RHS) != 0;
  if (i > m && fuse_delete_ok(c->variant) && (c->flags & AA_FUSE_DELETE) && c->k >= 2 &&
      c->k - 1 + (fuse_rhs ? 2 : 1) <= 64) {
    // QRDelete + QRAdd of Delta f_{i-1} with their first reductions merged
    s = fused_delete_add(c, c->W, fuse_rhs ? c->f_prev : nullptr, &rhs_done);
  } else {
    if (i > m) s = qr_delete_impl(c, true);  // Alg. 2: QRDelete when the window is full
    if (s == AA_OK)  // Alg. 2: QRAdd of Delta f_{i-1} (optionally also R gamma = Q^T f_i)
      s = qr_add_impl(c, c->W, fuse_rhs ? c->f_prev : nullptr, &rhs_done);
  }
  if (s == AA_OK && !rhs_done) s = rhs_impl(c, c->f_prev);  // R gamma = Q^T f_i
  if (s != AA_OK) return s;
  XupdArgs xa{c->ring, c->ldq, m, (int)((i - m_i) % m), m_i, g, x, x_next, c->n, c->sm.gamma};
  Tail tx = tail(TAIL_STEP, c->k);
  tx.m_i = m_i;
  if (timed(c, AA_K_XUPDATE, m_i + 3,
            [&] { return launch_xupdate(xa, c->sm, tx, G, st); }) != hipSuccess)
    return AA_EHIP;
  c->m_i = m_i;
  c->iter = i + 1;
  return AA_OK;
}

// With graphs on, a steady-state iteration (window full, grid-wide passes) is
// replayed from a HIP graph captured the first time its ring-slot phase comes
// round with these caller pointers; the host then only advances its counters
// by what the captured iteration did.
static aa_status step_graph(aa_ctx* c, const double* x, const double* g, double* x_next) {
  const int phase = (int)((c->iter - 1) % c->m);
  if ((int)c->graphs.size() != c->m) {
    drop_graphs(c);
    c->graphs.resize(c->m);
  }
  aa_ctx::StepGraph& sg = c->graphs[phase];
  if (sg.exec && sg.x == x && sg.g == g && sg.xn == x_next) {
    if (hipGraphLaunch(sg.exec, c->stream) != hipSuccess) return AA_EHIP;
    c->syncs_add += sg.d_add;
    c->syncs_del += sg.d_del;
    c->syncs_rhs += sg.d_rhs;
    c->m_i = c->m;
    c->iter += 1;
    return AA_OK;
  }
  if (sg.exec) {
    (void)hipGraphExecDestroy(sg.exec);
    sg.exec = nullptr;
  }
  const int64_t a0 = c->syncs_add, d0 = c->syncs_del, r0 = c->syncs_rhs;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return AA_EHIP;
  const aa_status s = step_enqueue(c, x, g, x_next);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &gr);
  if (s != AA_OK || e != hipSuccess || !gr) {
    if (gr) (void)hipGraphDestroy(gr);
    return s != AA_OK ? s : AA_EHIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (ei != hipSuccess) return AA_EHIP;
  sg.exec = exec;
  sg.x = x;
  sg.g = g;
  sg.xn = x_next;
  sg.d_add = c->syncs_add - a0;
  sg.d_del = c->syncs_del - d0;
  sg.d_rhs = c->syncs_rhs - r0;
  // the capture recorded the iteration (and advanced the host state); run it
  return hipGraphLaunch(exec, c->stream) == hipSuccess ? AA_OK : AA_EHIP;
}

aa_status aa_step(aa_ctx* c, const double* x, const double* g, double* x_next) {
  if (!c || !x || !g || !x_next || (c->flags & AA_QR_ONLY)) return AA_EINVAL;
  if (x_next == g) return AA_EINVAL;
  if (c->max_iter > 0 && c->iter > c->max_iter)  // the cap: iteration i = max_iter + 1 ends it
    return hip_ok(launch_stop_cap(c->stop_dev, c->k, c->m_i, x, x_next, c->n, c->stream));
  const bool one_wg = c->d_binst && c->n <= c->fused_max;
  if (c->graph_on && c->stream && !c->prof_on && !one_wg && c->iter > c->m && c->k == c->m)
    return step_graph(c, x, g, x_next);
  return step_enqueue(c, x, g, x_next);
}

aa_status aa_set_stop(aa_ctx* c, double tol, int64_t max_iter, int mode) {
  if (!c || !(tol == tol) || max_iter < 0 || (mode != AA_STOP_RESIDUAL && mode != AA_STOP_STEP))
    return AA_EINVAL;
  drop_graphs(c);  // captured iterations carry the test in their launch arguments
  c->stop_tol = tol > 0.0 ? tol : 0.0;
  c->stop_mode = tol > 0.0 ? (mode == AA_STOP_STEP ? kStopStep : kStopResidual) : kStopNone;
  c->max_iter = max_iter;
  return AA_OK;
}

aa_status aa_set_graph(aa_ctx* c, int enable) {
  if (!c) return AA_EINVAL;
  if (enable && !c->stream) return AA_EINVAL;  // capture needs a stream of its own
  c->graph_on = enable != 0;
  if (!c->graph_on) drop_graphs(c);
  return AA_OK;
}

aa_status aa_get_info(aa_ctx* c, aa_info* info) {
  if (!c || !info) return AA_EINVAL;
  double sc[S_COUNT];
  int status = 0;
  StopState stop{};
  if (hipMemcpyAsync(sc, c->sm.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return AA_EHIP;
  if (hipMemcpyAsync(&status, c->sm.status, sizeof(int), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return AA_EHIP;
  if (hipMemcpyAsync(&stop, c->stop_dev, sizeof(stop), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return AA_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return AA_EHIP;
  if (stop.done != 0) {
    // steps enqueued after the end changed nothing on the device: report (and
    // resume counting from) the state in which the iteration ended
    drop_graphs(c);
    c->iter = stop.iter;
    c->k = stop.k;
    c->m_i = stop.m_i;
  }
  info->stopped = stop.done;
  info->stop_iter = stop.done ? stop.iter : -1;
  info->iter = c->iter;
  info->m_i = c->m_i;
  info->k = c->k;
  info->res_norm = sqrt(sc[S_RES]);
  info->res0_norm = sqrt(sc[S_RES0]);
  info->step_norm = sqrt(sc[S_STEP]);
  info->status = status;
  return AA_OK;
}

aa_status aa_qr_add(aa_ctx* c, const double* v) {
  if (!c || !v) return AA_EINVAL;
  return qr_add_impl(c, v);
}

aa_status aa_qr_delete(aa_ctx* c) {
  if (!c) return AA_EINVAL;
  return qr_delete_impl(c, false);
}

aa_status aa_qr_solve(aa_ctx* c, const double* f, double* gamma) {
  if (!c || !f || !gamma) return AA_EINVAL;
  if (c->k == 0) return AA_ESTATE;
  if (c->k > 64) return AA_EINVAL;  // the back substitution runs on one 64-lane wave
  aa_status s = rhs_impl(c, f);
  if (s != AA_OK) return s;
  return hip_ok(launch_copy(gamma, c->sm.gamma, c->k, c->stream));
}

aa_status aa_get_qr(aa_ctx* c, double* hR, double* hT, int* k) {
  if (!c) return AA_EINVAL;
  const int kk = c->k, cap = c->sm.cap;
  if (k) *k = kk;
  if (kk == 0) return hip_ok(hipStreamSynchronize(c->stream));
  if (hR && hipMemcpy2DAsync(hR, kk * sizeof(double), c->sm.R, cap * sizeof(double),
                             kk * sizeof(double), kk, hipMemcpyDeviceToHost,
                             c->stream) != hipSuccess)
    return AA_EHIP;
  if (hT && hipMemcpy2DAsync(hT, kk * sizeof(double), c->sm.T, cap * sizeof(double),
                             kk * sizeof(double), kk, hipMemcpyDeviceToHost,
                             c->stream) != hipSuccess)
    return AA_EHIP;
  return hip_ok(hipStreamSynchronize(c->stream));
}

aa_status aa_qr_basis(aa_ctx* c, double** dQ, int64_t* ldq) {
  if (!c || !dQ || !ldq) return AA_EINVAL;
  *dQ = c->Q;
  *ldq = c->ldq;
  return AA_OK;
}

aa_status aa_qr_load(aa_ctx* c, int k, const double* dQ, int64_t ldq, const double* hR,
                     const double* hT) {
  if (c) drop_graphs(c);
  if (!c || k < 0 || k > c->cap || (k > 0 && (!dQ || !hR)) || ldq < c->n) return AA_EINVAL;
  const int cap = c->sm.cap;
  if (k > 0) {
    if (hipMemcpy2DAsync(c->Q, c->ldq * sizeof(double), dQ, ldq * sizeof(double),
                         c->n * sizeof(double), k, hipMemcpyDeviceToDevice,
                         c->stream) != hipSuccess)
      return AA_EHIP;
    // full cap x cap images so that entries outside the k x k block are zero
    double* R = (double*)calloc((size_t)cap * cap, sizeof(double));
    double* T = (double*)calloc((size_t)cap * cap, sizeof(double));
    if (!R || !T) {
      free(R);
      free(T);
      return AA_EINVAL;
    }
    for (int j = 0; j < cap; ++j) T[j + (size_t)j * cap] = 1.0;
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) {
        R[i + (size_t)j * cap] = hR[i + (size_t)j * k];
        if (hT && i != j) T[i + (size_t)j * cap] = hT[i + (size_t)j * k];
      }
    hipError_t e1 = hipMemcpyAsync(c->sm.R, R, sizeof(double) * cap * cap,
                                   hipMemcpyHostToDevice, c->stream);
    hipError_t e2 = hipMemcpyAsync(c->sm.T, T, sizeof(double) * cap * cap,
                                   hipMemcpyHostToDevice, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    free(R);
    free(T);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return AA_EHIP;
  }
  c->k = k;
  return AA_OK;
}

aa_status aa_reset(aa_ctx* c) {
  if (c) drop_graphs(c);
  if (!c) return AA_EINVAL;
  c->iter = 0;
  c->k = 0;
  c->m_i = 0;
  Small s0 = c->sm;
  s0.stop = c->stop_dev;
  return hip_ok(launch_init_small(s0, c->stream));
}

aa_status aa_destroy(aa_ctx* c) {
  if (!c) return AA_OK;
  drop_graphs(c);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
  return AA_OK;
}

aa_status aa_profile_enable(aa_ctx* c, int enable) {
  if (!c) return AA_EINVAL;
  if (enable && c->ev.empty()) {
    c->ev.resize(3 * kEventPairs);
    c->ev_kind.resize(kEventPairs);
    c->ev_mid.resize(kEventPairs);
    for (auto& e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return AA_EHIP;
  }
  c->prof_on = enable != 0;
  return aa_profile_reset(c);
}

aa_status aa_profile_reset(aa_ctx* c) {
  if (!c) return AA_EINVAL;
  if (c->ev_used && hipStreamSynchronize(c->stream) != hipSuccess) return AA_EHIP;
  c->ev_used = 0;
  for (int k = 0; k < AA_K_COUNT; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_launches[k] = 0;
    c->prof_bytes[k] = 0.0;
  }
  return AA_OK;
}

aa_status aa_profile_read(aa_ctx* c, int kind, double* ms, int64_t* launches, double* bytes) {
  if (!c || kind < 0 || kind >= AA_K_COUNT) return AA_EINVAL;
  if (prof_drain(c) != hipSuccess) return AA_EHIP;
  if (ms) *ms = c->prof_ms[kind];
  if (launches) *launches = c->prof_launches[kind];
  if (bytes) *bytes = c->prof_bytes[kind];
  return AA_OK;
}

aa_status aa_set_fused_threshold(aa_ctx* c, int64_t n_max) {
  if (c) drop_graphs(c);
  if (!c || n_max < 0) return AA_EINVAL;
  c->fused_max = c->one_wg_ok ? n_max : 0;
  return AA_OK;
}

aa_status aa_set_grid(aa_ctx* c, int stream_max, int gram_max) {
  if (c) drop_graphs(c);
  if (!c || stream_max < 1 || stream_max > 4096 || gram_max < 1 || gram_max > 4096)
    return AA_EINVAL;
  // every pass publishes (values reduced) x (workgroups) partials; the Gram
  // pass clamps its grid to the partials buffer by itself
  if ((size_t)stream_max * kMaxRed > kPartials) return AA_EINVAL;
  c->grid_stream_max = stream_max;
  c->grid_gram_max = gram_max;
  return AA_OK;
}

aa_status aa_sync_counts(aa_ctx* c, int64_t* add, int64_t* del, int64_t* rhs) {
  if (!c) return AA_EINVAL;
  if (add) *add = c->syncs_add;
  if (del) *del = c->syncs_del;
  if (rhs) *rhs = c->syncs_rhs;
  return AA_OK;
}

aa_status aa_problem_apply(int dim, int64_t s, double h, double omega, double c,
                           const double* f, const double* u, double* out, void* stream) {
  if (dim < 1 || dim > 3 || s < 1 || !f || !u || !out || u == out || !(h > 0.0))
    return AA_EINVAL;
  return hip_ok(launch_stencil(dim, s, h, omega, c, f, u, out, (hipStream_t)stream));
}

aa_status aa_fill_uniform(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                          uint64_t offset, double lo, double hi, void* stream) {
  if (!out || n < 0) return AA_EINVAL;
  if (n == 0) return AA_OK;
  return hip_ok(launch_fill_uniform(out, n, seed, stream_id, offset, lo, hi, (hipStream_t)stream));
}

aa_status aa_fill_normal(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                         uint64_t offset, void* stream) {
  if (!out || n < 0) return AA_EINVAL;
  if (n == 0) return AA_OK;
  return hip_ok(launch_fill_normal(out, n, seed, stream_id, offset, (hipStream_t)stream));
}

aa_status aa_em_apply(const aa_em_mixture* mix, const double* x, int64_t nsamples,
                      const double* u, double* out, int64_t n, double* work, void* stream) {
  if (!mix || !x || !u || !out || !work || nsamples < 1 || n < 3 || n % 3 != 0)
    return AA_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(mix->alpha[i] > 0.0) || !(mix->sigma[i] > 0.0)) return AA_EINVAL;
  return hip_ok(launch_em(mix->alpha, mix->sigma, x, nsamples, u, out, n, work,
                          (hipStream_t)stream));
}

aa_status aa_bandwidth_probe(int reads, int writes, const double* src, int64_t ld, double* dst,
                             int64_t n, double* sink, void* stream) {
  if (n < 1 || ld < n || !src || (writes > 0 && !dst) || (writes == 0 && !sink)) return AA_EINVAL;
  int64_t g = (n + kTile - 1) / kTile;
  const int grid = (int)(g > 1024 ? 1024 : g);
  const hipError_t e =
      launch_probe(reads, writes, src, ld, dst, n, sink, grid, (hipStream_t)stream);
  return e == hipErrorInvalidValue ? AA_EINVAL : hip_ok(e);
}

const char* aa_version(void) { return "aa-mi355x 0.1 (gfx950, fp64)"; }

}  // extern "C"
