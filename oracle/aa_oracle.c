/*
 * aa_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for Anderson
 * acceleration with the QR-update variants of Lockhart, Gardner, Woodward,
 * Thomas and Olson, "Performance of Low Synchronization Orthogonalization
 * Methods in Anderson Accelerated Fixed Point Solvers" (arXiv 2110.09667).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the HIP library.
 *
 * Conventions (Sec. 3 of the paper): 0-based indices, inclusive slices.
 *   Q  -- n x cap, column-major, leading dimension ld (column j at Q + j*ld)
 *   R  -- cap x cap, column-major (R[i + j*cap]), upper triangular
 *   T  -- cap x cap, column-major, unit lower triangular (ICWY only)
 *   k  -- number of columns currently held in Q (k = m_i - 1 when QRAdd
 *         starts, k = m_i when it returns)
 *
 * Arithmetic: IEEE FP64, round to nearest, compiled with -ffp-contract=off so
 * no multiply-add is fused.  Dot products and norms use Neumaier-compensated
 * summation, so the oracle is at least as accurate as any GPU summation order.
 * No fusion or reordering beyond what the algorithms state.  A dot product
 * sums fixed blocks of OR_BLOCK rows (each compensated), then the block
 * results in block order (compensated again): the same source built with
 * OpenMP (-fopenmp, the CPU baseline) runs the blocks and the elementwise row
 * loops on several threads and gives bitwise the same results as the
 * single-threaded build, whatever the thread count.
 *
 * "Sync" counters: every global reduction the paper marks (Algs. 3-6 and the
 * ICWY refresh of T after QRDelete, Sec. 3.2) increments a counter, so tests
 * can check the counts of Sec. 4.1.  The right-hand side Q^T f_i of the LSP
 * solve (Alg. 2) is counted separately: the paper's totals do not include it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* OR_DCGS2_LAG: the delayed CGS-2 with the normalization lagged as well
 * (Sec. 3.4 describes it in words, after Swirydowicz et al. and Bielich et
 * al.; the paper does not use it in AA). */
enum { OR_MGS = 0, OR_CGS2 = 1, OR_DCGS2 = 2, OR_ICWY = 3, OR_DCGS2_LAG = 4 };

/* Readings of passages the paper leaves open (listed in the design notes). */
enum {
  OR_DCGS2_LITERAL = 1u << 1, /* Alg. 6: add s itself (not R_kk*s) to R      */
  OR_ICWY_T_TRANSFORM = 1u << 2, /* ICWY: T after QRDelete by rotating the
                                    old Gram matrix, no reduction (Sec. 3.2) */
  OR_DCGS2_GUARD_GE3 = 1u << 4 /* Alg. 6: reorthogonalize when m_i >= 3      */
};

enum { OR_OK = 0, OR_EINVAL = -1, OR_EBREAKDOWN = -3, OR_ESTATE = -4 };

/* ------------------------------------------------------------------ */
/* vector primitives                                                   */
/* ------------------------------------------------------------------ */

#ifdef _OPENMP
#include <omp.h>
#define OR_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PARALLEL_FOR
#endif

/* Rows per block of a dot product (the unit of work of a thread). */
#define OR_BLOCK 65536

/* Neumaier's compensated accumulation of p into (s, comp). */
static inline void neumaier_add(double *s, double *comp, double p) {
  double t = *s + p;
  if (fabs(*s) >= fabs(p))
    *comp += (*s - t) + p;
  else
    *comp += (p - t) + *s;
  *s = t;
}

/* x^T y (or (x - y)^T (x - y) with diff) over rows [r0, r1), compensated. */
static double block_dot(int64_t r0, int64_t r1, const double *x, const double *y, int diff) {
  double s = 0.0, comp = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    double p;
    if (diff) {
      double d = x[r] - y[r];
      p = d * d;
    } else {
      p = x[r] * y[r];
    }
    neumaier_add(&s, &comp, p);
  }
  return s + comp;
}

/* Compensated sum of the block results in block order. */
static double blocked_sum(int64_t n, const double *x, const double *y, int diff) {
  int64_t nb = (n + OR_BLOCK - 1) / OR_BLOCK;
  if (nb <= 1) return block_dot(0, n, x, y, diff);
  double *part = (double *)malloc(sizeof(double) * (size_t)nb);
  OR_PARALLEL_FOR
  for (int64_t b = 0; b < nb; ++b) {
    int64_t r1 = (b + 1) * OR_BLOCK;
    part[b] = block_dot(b * OR_BLOCK, r1 < n ? r1 : n, x, y, diff);
  }
  double s = 0.0, comp = 0.0;
  for (int64_t b = 0; b < nb; ++b) neumaier_add(&s, &comp, part[b]);
  free(part);
  return s + comp;
}

/* x^T y with Neumaier's compensated summation of the rounded products. */
static double dot(int64_t n, const double *x, const double *y) { return blocked_sum(n, x, y, 0); }

/* ||x - y||_2^2, compensated. */
static double sqdist(int64_t n, const double *x, const double *y) {
  return blocked_sum(n, x, y, 1);
}

static double nrm2(int64_t n, const double *x) { return sqrt(dot(n, x, x)); }

/* y <- y - a x */
static void axmy(int64_t n, double a, const double *x, double *y) {
  OR_PARALLEL_FOR
  for (int64_t r = 0; r < n; ++r) y[r] = y[r] - a * x[r];
}

/* Threads of the OpenMP build (the CPU baseline); a no-op without OpenMP.
 * Returns the thread count in effect. */
int or_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
  return omp_get_max_threads();
#else
  (void)t;
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* the QR factorization of F_i                                         */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t n;   /* rows */
  int64_t ld;  /* leading dimension of Q (>= n) */
  int cap;     /* column capacity of Q, R, T */
  int k;       /* columns currently in Q */
  double *Q;   /* ld x cap */
  double *R;   /* cap x cap */
  double *T;   /* cap x cap */
  double *work;/* 2*n scratch */
  int64_t syncs_add, syncs_delete, syncs_rhs;
} or_qr;

#define QCOL(s, j) ((s)->Q + (int64_t)(j) * (s)->ld)
#define RM(s, i, j) ((s)->R[(i) + (int64_t)(j) * (s)->cap])
#define TM(s, i, j) ((s)->T[(i) + (int64_t)(j) * (s)->cap])

/* Breakdown: the new column's R_kk at most 64 eps times the norm of its
 * column of R (the column numerically in the span of the window; the paper
 * does not treat rank deficiency, reading A10). */
#define OR_BREAKDOWN_REL (64.0 * 2.220446049250313e-16)

/* Final normalization shared by every QRAdd variant (last two lines of
 * Algs. 3-6): R_kk = ||v||_2 (one Sync), q_k = v / R_kk. */
static int normalize_into(or_qr *s, double *v) {
  int k = s->k;
  double nv = nrm2(s->n, v);
  s->syncs_add += 1;
  RM(s, k, k) = nv;
  double col = nv * nv;
  for (int j = 0; j < k; ++j) col += RM(s, j, k) * RM(s, j, k);
  if (!(nv > OR_BREAKDOWN_REL * sqrt(col)) || !isfinite(nv)) return OR_EBREAKDOWN;
  double *q = QCOL(s, k);
  OR_PARALLEL_FOR
  for (int64_t r = 0; r < s->n; ++r) q[r] = v[r] / nv;
  s->k = k + 1;
  return OR_OK;
}

/* Alg. 3, QRAdd_MGS: orthogonalize v against q_0..q_{k-1} one column at a
 * time; each coefficient is its own reduction (k Syncs), then normalize. */
static int qr_add_mgs(or_qr *s, double *v) {
  int k = s->k;
  for (int j = 0; j < k; ++j) {
    double rj = dot(s->n, QCOL(s, j), v);
    s->syncs_add += 1;
    RM(s, j, k) = rj;
    axmy(s->n, rj, QCOL(s, j), v);
  }
  return normalize_into(s, v);
}

/* Alg. 5, QRAdd_CGS2: classical Gram-Schmidt applied twice.
 * s = Q^T v (Sync); y = v - Q s; z = Q^T y (Sync); v = y - Q z; R = s + z. */
static int qr_add_cgs2(or_qr *s, double *v) {
  int k = s->k;
  if (k > 0) {
    double *sc = (double *)malloc(sizeof(double) * (size_t)k);
    double *zc = (double *)malloc(sizeof(double) * (size_t)k);
    for (int j = 0; j < k; ++j) sc[j] = dot(s->n, QCOL(s, j), v);
    s->syncs_add += 1;
    for (int j = 0; j < k; ++j) axmy(s->n, sc[j], QCOL(s, j), v); /* v is y */
    for (int j = 0; j < k; ++j) zc[j] = dot(s->n, QCOL(s, j), v);
    s->syncs_add += 1;
    for (int j = 0; j < k; ++j) axmy(s->n, zc[j], QCOL(s, j), v);
    for (int j = 0; j < k; ++j) RM(s, j, k) = sc[j] + zc[j];
    free(sc);
    free(zc);
  }
  return normalize_into(s, v);
}

/* Alg. 4, QRAdd_ICWY (inverse compact WY MGS, two reductions):
 * row k-1 of the unit lower triangular T holds q_{k-1}^T q_b for b < k-1;
 * it is computed in the same reduction as r = Q^T v.  Then T r' = r is
 * solved by forward substitution and v = v - Q r'. */
static int qr_add_icwy(or_qr *s, double *v) {
  int k = s->k;
  if (k > 0) {
    double *rc = (double *)malloc(sizeof(double) * (size_t)k);
    const double *qlast = QCOL(s, k - 1);
    for (int b = 0; b < k - 1; ++b) TM(s, k - 1, b) = dot(s->n, QCOL(s, b), qlast);
    for (int j = 0; j < k; ++j) rc[j] = dot(s->n, QCOL(s, j), v);
    s->syncs_add += 1; /* the delayed Sync and the Sync are one reduction */
    TM(s, k - 1, k - 1) = 1.0;
    /* forward substitution with the unit lower triangle T_{0:k-1,0:k-1} */
    for (int a = 0; a < k; ++a) {
      double acc = rc[a];
      for (int b = 0; b < a; ++b) acc -= TM(s, a, b) * rc[b];
      rc[a] = acc;
    }
    for (int j = 0; j < k; ++j) RM(s, j, k) = rc[j];
    for (int j = 0; j < k; ++j) axmy(s->n, rc[j], QCOL(s, j), v);
    free(rc);
  }
  TM(s, k, k) = 1.0;
  return normalize_into(s, v);
}

/* Alg. 6, QRAdd_DCGS2 (delayed reorthogonalization, two reductions).
 * R_{0:k-1,k} = Q^T v with the current q_{k-1} (delayed Sync).  If m_i > 3,
 * in the same reduction s = Q_{:,0:k-2}^T q_{k-1}; then q_{k-1} is
 * reorthogonalized, q_{k-1} -= Q_{:,0:k-2} s, and column k-1 of R is
 * corrected so that Q R = F_i still holds: R_{0:k-2,k-1} += R_{k-1,k-1} s
 * (the literal reading adds s itself).  Finally v -= Q_{:,0:k-1} R_{0:k-1,k}
 * using the reorthogonalized q_{k-1}; q_{k-1} is not renormalized. */
static int qr_add_dcgs2(or_qr *s, double *v, unsigned flags) {
  int k = s->k;
  int m_i = k + 1;
  if (k > 0) {
    for (int j = 0; j < k; ++j) RM(s, j, k) = dot(s->n, QCOL(s, j), v);
    int reorth = (flags & OR_DCGS2_GUARD_GE3) ? (m_i >= 3) : (m_i > 3);
    if (reorth) {
      int p = k - 1; /* the previous column, index m_i - 2 */
      double *sc = (double *)malloc(sizeof(double) * (size_t)p);
      for (int j = 0; j < p; ++j) sc[j] = dot(s->n, QCOL(s, j), QCOL(s, p));
      s->syncs_add += 1; /* shared with the delayed Sync above */
      for (int j = 0; j < p; ++j) axmy(s->n, sc[j], QCOL(s, j), QCOL(s, p));
      double scale = (flags & OR_DCGS2_LITERAL) ? 1.0 : RM(s, p, p);
      for (int j = 0; j < p; ++j) RM(s, j, p) = RM(s, j, p) + scale * sc[j];
      free(sc);
    } else {
      s->syncs_add += 1; /* the delayed Sync alone */
    }
    for (int j = 0; j < k; ++j) axmy(s->n, RM(s, j, k), QCOL(s, j), v);
  }
  return normalize_into(s, v);
}

/* DCGS-2 with the normalization lagged (Sec. 3.4, the stable form the paper
 * describes but does not run in AA: the correction matrix I - L - L^T split
 * into I - L, applied when a column is added, and L^T, applied one add
 * later, with the new column's normalization lagged too).  Invariant: columns
 * 0..k-2 are final; column k-1 (the newest) has been orthogonalized once and
 * scaled by a norm obtained from Pythagoras, not from a reduction over it.
 *
 * Adding v (k >= 1 columns present, p = k-1 the newest), ONE reduction:
 *   s = Q_{0:p-1}^T q_p,  z = Q_{0:p-1}^T v,
 *   alpha = q_p^T q_p,    beta = q_p^T v,    nu = v^T v.
 * Delayed reorthogonalization and normalization of q_p:
 *   rho = sqrt(alpha - s^T s),  q_p <- (q_p - Q_{0:p-1} s) / rho,
 *   and column p of R follows so that Q R = F keeps holding:
 *   R_{0:p-1,p} += R_pp s,  R_pp <- rho R_pp.
 * Projection of v on the updated basis (once; its reorthogonalization waits
 * for the next add):  R_{0:p-1,k} = z,  R_pk = (beta - s^T z) / rho,
 *   w = v - Q_{0:p-1} z - q_p R_pk,
 *   R_kk = sqrt(nu - ||R_{0:p,k}||^2)   (Pythagoras: no reduction over w),
 *   q_k = w / R_kk.
 * With k = 0 the column is normalized by its explicit norm (one reduction).
 * A non-positive alpha - s^T s or nu - ||R_{0:p,k}||^2 (cancellation when v
 * is nearly in the span of Q) is a breakdown. */
static int qr_add_dcgs2_lag(or_qr *s, double *v) {
  int k = s->k;
  if (k == 0) return normalize_into(s, v);
  int p = k - 1;
  int64_t n = s->n;
  double *qp = QCOL(s, p);
  double *sc = (double *)calloc((size_t)k, sizeof(double));
  double *zc = (double *)calloc((size_t)k, sizeof(double));
  for (int j = 0; j < p; ++j) {
    sc[j] = dot(n, QCOL(s, j), qp);
    zc[j] = dot(n, QCOL(s, j), v);
  }
  double alpha = dot(n, qp, qp), beta = dot(n, qp, v), nu = dot(n, v, v);
  s->syncs_add += 1; /* all five in one reduction */
  double ss = 0.0, sz = 0.0;
  for (int j = 0; j < p; ++j) {
    ss += sc[j] * sc[j];
    sz += sc[j] * zc[j];
  }
  double rho2 = alpha - ss;
  int st = OR_OK;
  if (!(rho2 > OR_BREAKDOWN_REL * alpha) || !isfinite(rho2)) {
    st = OR_EBREAKDOWN;
  } else {
    double rho = sqrt(rho2);
    for (int j = 0; j < p; ++j) axmy(n, sc[j], QCOL(s, j), qp);
    OR_PARALLEL_FOR
    for (int64_t r = 0; r < n; ++r) qp[r] = qp[r] / rho;
    double rpp = RM(s, p, p);
    for (int j = 0; j < p; ++j) RM(s, j, p) = RM(s, j, p) + rpp * sc[j];
    RM(s, p, p) = rho * rpp;
    double rpk = (beta - sz) / rho;
    double rr = 0.0;
    for (int j = 0; j < p; ++j) {
      RM(s, j, k) = zc[j];
      rr += zc[j] * zc[j];
    }
    RM(s, p, k) = rpk;
    rr += rpk * rpk;
    double w2 = nu - rr;
    double rkk = sqrt(w2);
    /* nu - ||r||^2 carries rounding of order eps nu: below 64 eps nu the
     * new column's norm is noise (it is numerically in the span) */
    if (!(w2 > OR_BREAKDOWN_REL * nu) || !isfinite(w2)) {
      st = OR_EBREAKDOWN;
    } else {
      for (int j = 0; j < p; ++j) axmy(n, zc[j], QCOL(s, j), v);
      axmy(n, rpk, qp, v);
      RM(s, k, k) = rkk;
      double *q = QCOL(s, k);
      OR_PARALLEL_FOR
      for (int64_t r = 0; r < n; ++r) q[r] = v[r] / rkk;
      s->k = k + 1;
    }
  }
  free(sc);
  free(zc);
  return st;
}

/* The lagged DCGS-2's last step on its own: reorthogonalize and renormalize
 * the newest column (one reduction, as the paper notes the last iteration of
 * the lagged form needs), so that every column is final. */
int or_qr_flush(or_qr *s, int variant) {
  if (variant != OR_DCGS2_LAG) return OR_EINVAL;
  int k = s->k;
  if (k == 0) return OR_OK;
  int p = k - 1;
  int64_t n = s->n;
  double *qp = QCOL(s, p);
  double *sc = (double *)calloc((size_t)k, sizeof(double));
  for (int j = 0; j < p; ++j) sc[j] = dot(n, QCOL(s, j), qp);
  double alpha = dot(n, qp, qp);
  s->syncs_add += 1;
  double ss = 0.0;
  for (int j = 0; j < p; ++j) ss += sc[j] * sc[j];
  double rho2 = alpha - ss;
  int st = OR_OK;
  if (!(rho2 > OR_BREAKDOWN_REL * alpha) || !isfinite(rho2)) {
    st = OR_EBREAKDOWN;
  } else {
    double rho = sqrt(rho2);
    for (int j = 0; j < p; ++j) axmy(n, sc[j], QCOL(s, j), qp);
    OR_PARALLEL_FOR
    for (int64_t r = 0; r < n; ++r) qp[r] = qp[r] / rho;
    double rpp = RM(s, p, p);
    for (int j = 0; j < p; ++j) RM(s, j, p) = RM(s, j, p) + rpp * sc[j];
    RM(s, p, p) = rho * rpp;
  }
  free(sc);
  return st;
}

/* Alg. 2, QRAdd: append v (not modified) as column k of the factorization. */
int or_qr_add(or_qr *s, int variant, unsigned flags, const double *v_in) {
  if (s->k >= s->cap) return OR_ESTATE;
  double *v = s->work;
  memcpy(v, v_in, sizeof(double) * (size_t)s->n);
  for (int j = 0; j <= s->k; ++j) RM(s, j, s->k) = 0.0;
  switch (variant) {
    case OR_MGS: return qr_add_mgs(s, v);
    case OR_CGS2: return qr_add_cgs2(s, v);
    case OR_DCGS2: return qr_add_dcgs2(s, v, flags);
    case OR_ICWY: return qr_add_icwy(s, v);
    case OR_DCGS2_LAG: return qr_add_dcgs2_lag(s, v);
    default: return OR_EINVAL;
  }
}

/* Alg. 2, QRDelete: drop column 0 of F_i and restore the factorization with
 * Givens rotations (the paper names the method, Sec. 2.1 and 3.2, but does
 * not print it; this is the textbook form).
 *
 * H = R_{:,1:k-1} is upper Hessenberg (k x (k-1)).  For j = 0..k-2 the
 * rotation G_j = [c s; -s c] with rho = hypot(a, b), c = a/rho, s = b/rho,
 * (a, b) = (H_jj, H_{j+1,j}), zeroes H_{j+1,j}; it is applied to rows j, j+1
 * of H and, transposed, to columns j, j+1 of Q so that Q H is unchanged:
 *   q_j <- c q_j + s q_{j+1},   q_{j+1} <- -s q_j + c q_{j+1}.
 * rho >= 0 keeps the diagonal of the new R nonnegative, so the result is the
 * unique QR of the retained columns.  The last row of H and the last column
 * of Q are then dropped.  No reduction is needed, except that ICWY must
 * refresh T (Sec. 3.2): T_ab = q_a^T q_b for b < a, T_aa = 1, recomputed
 * over the rotated columns in one reduction.
 *
 * With OR_ICWY_T_TRANSFORM the refresh needs no reduction: the old Gram
 * matrix S = I + L + L^T (L the strict lower part of T) is rotated like the
 * columns of Q, S <- W^T S W with the same rotations, and its strict lower
 * part is the new T.  The new columns 0..k-3 are combinations of the old
 * columns 0..k-2 only (rotation j leaves column j final), whose rows of T
 * are current, so rotations 0..k-3 applied to the leading (k-1) x (k-1)
 * block of S give rows 0..k-3 of the new T exactly.  The last row (the
 * newest retained column, which old column k-1 entered) is the Gram row the
 * next QRAdd's first reduction computes before anything reads it (Alg. 4);
 * it is zeroed here. */
int or_qr_delete(or_qr *s, int variant, unsigned flags) {
  int k = s->k;
  if (k <= 0) return OR_ESTATE;
  if (k == 1) {
    s->k = 0;
    RM(s, 0, 0) = 0.0;
    return OR_OK;
  }
  int transform = variant == OR_ICWY && (flags & OR_ICWY_T_TRANSFORM);
  int kk = k - 1;
  double *S = NULL, *gc = NULL, *gs = NULL;
  if (transform) {
    S = (double *)calloc((size_t)kk * (size_t)kk, sizeof(double));
    gc = (double *)calloc((size_t)kk, sizeof(double));
    gs = (double *)calloc((size_t)kk, sizeof(double));
    for (int a = 0; a < kk; ++a) {
      S[a + (int64_t)a * kk] = 1.0;
      for (int b = 0; b < a; ++b) {
        S[a + (int64_t)b * kk] = TM(s, a, b);
        S[b + (int64_t)a * kk] = TM(s, a, b);
      }
    }
  }
  /* shift R left by one column: H_{:,j} = R_{:,j+1} */
  for (int j = 0; j < k - 1; ++j)
    for (int i = 0; i < k; ++i) RM(s, i, j) = RM(s, i, j + 1);
  for (int i = 0; i < k; ++i) RM(s, i, k - 1) = 0.0;
  for (int j = 0; j < k - 1; ++j) {
    double a = RM(s, j, j), b = RM(s, j + 1, j);
    double rho = hypot(a, b);
    double c = 1.0, sn = 0.0;
    if (rho > 0.0) {
      c = a / rho;
      sn = b / rho;
    }
    for (int col = j; col < k - 1; ++col) {
      double hj = RM(s, j, col), hj1 = RM(s, j + 1, col);
      RM(s, j, col) = c * hj + sn * hj1;
      RM(s, j + 1, col) = -sn * hj + c * hj1;
    }
    RM(s, j + 1, j) = 0.0;
    if (transform) {
      gc[j] = c;
      gs[j] = sn;
    }
    double *qa = QCOL(s, j), *qb = QCOL(s, j + 1);
    OR_PARALLEL_FOR
    for (int64_t r = 0; r < s->n; ++r) {
      double x = qa[r], y = qb[r];
      qa[r] = c * x + sn * y;
      qb[r] = -sn * x + c * y;
    }
  }
  for (int i = 0; i < k; ++i) RM(s, k - 1, i) = 0.0;
  s->k = k - 1;
  if (transform) {
    /* S <- W^T S W, rotations 0..kk-2 (columns j, j+1, then rows j, j+1) */
#define SM(i, j) S[(i) + (int64_t)(j) * kk]
    for (int j = 0; j + 1 < kk; ++j) {
      double c = gc[j], sn = gs[j];
      for (int r = 0; r < kk; ++r) {
        double x = SM(r, j), y = SM(r, j + 1);
        SM(r, j) = c * x + sn * y;
        SM(r, j + 1) = -sn * x + c * y;
      }
      for (int r = 0; r < kk; ++r) {
        double x = SM(j, r), y = SM(j + 1, r);
        SM(j, r) = c * x + sn * y;
        SM(j + 1, r) = -sn * x + c * y;
      }
    }
    for (int a = 0; a < kk; ++a) {
      for (int b = 0; b < a; ++b) TM(s, a, b) = (a < kk - 1) ? SM(a, b) : 0.0;
      TM(s, a, a) = 1.0;
      for (int b = a + 1; b < s->cap; ++b) TM(s, a, b) = 0.0;
    }
#undef SM
    free(S);
    free(gc);
    free(gs);
  } else if (variant == OR_ICWY) {
    for (int a = 0; a < s->k; ++a) {
      for (int b = 0; b < a; ++b) TM(s, a, b) = dot(s->n, QCOL(s, b), QCOL(s, a));
      TM(s, a, a) = 1.0;
      for (int b = a + 1; b < s->cap; ++b) TM(s, a, b) = 0.0;
    }
    s->syncs_delete += 1;
  }
  return OR_OK;
}

/* Alg. 2, last line, right-hand side: c = Q^T f (one reduction). */
void or_qr_rhs(or_qr *s, const double *f, double *c) {
  for (int j = 0; j < s->k; ++j) c[j] = dot(s->n, QCOL(s, j), f);
  s->syncs_rhs += 1;
}

/* Back substitution R gamma = c for the k x k upper triangle. */
int or_backsolve(int k, int cap, const double *R, const double *c, double *gamma) {
  for (int a = k - 1; a >= 0; --a) {
    double acc = c[a];
    for (int b = a + 1; b < k; ++b) acc -= R[a + (int64_t)b * cap] * gamma[b];
    double d = R[a + (int64_t)a * cap];
    if (!(d != 0.0) || !isfinite(d)) return OR_EBREAKDOWN;
    gamma[a] = acc / d;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Anderson acceleration, Alg. 1 with the LSP solve of Alg. 2          */
/* ------------------------------------------------------------------ */

typedef struct {
  or_qr qr;
  int m;           /* window */
  int variant;
  unsigned flags;
  int64_t i;       /* index of the next iteration (0 before the first call) */
  int m_i;         /* columns used by the last step */
  double *f_prev;  /* f_{i-1} (n) */
  double *g_prev;  /* G(x_{i-1}) (n) */
  double *dG;      /* ring of Delta g, ld x m, Delta g_k in slot k mod m */
  double *dF;      /* ring of raw Delta f, ld x m (kept only for checks) */
  double *gamma;   /* m */
  double *c;       /* m, Q^T f_i */
  double *f;       /* n, f_i of the last step */
  double res_norm; /* ||f_i||_2 of the last step */
  double res0_norm;/* ||f_0||_2 */
  double step_norm;/* ||x_{i+1} - x_i||_2 of the last step */
  int status;
} or_aa;

/* One iteration of Alg. 1.  On the first call (i = 0) it returns
 * x_1 = G(x_0) and stores f_0 = G(x_0) - x_0.  On call i >= 1, given x_i and
 * g = G(x_i), it forms f_i, Delta f_{i-1}, Delta g_{i-1}, updates the QR of
 * F_i (Alg. 2: QRDelete when i > m, then QRAdd; at i = 1 the first column is
 * just normalized), solves R gamma = Q^T f_i and returns
 * x_{i+1} = G(x_i) - sum_j gamma_j Delta g_{i-m_i+j}. */
int or_aa_step(or_aa *a, const double *x, const double *g, double *x_next) {
  or_qr *s = &a->qr;
  int64_t n = s->n;
  if (a->i == 0) {
    OR_PARALLEL_FOR
    for (int64_t r = 0; r < n; ++r) {
      a->f_prev[r] = g[r] - x[r];
      a->g_prev[r] = g[r];
      x_next[r] = g[r];
    }
    memcpy(a->f, a->f_prev, sizeof(double) * (size_t)n);
    a->res0_norm = a->res_norm = nrm2(n, a->f_prev);
    a->step_norm = sqrt(sqdist(n, x_next, x));
    a->m_i = 0;
    a->i = 1;
    return OR_OK;
  }
  int64_t i = a->i;
  int m = a->m;
  int m_i = (int)(i < m ? i : m);
  int slot = (int)((i - 1) % m);
  double *df = a->dF + (int64_t)slot * s->ld;
  double *dg = a->dG + (int64_t)slot * s->ld;
  OR_PARALLEL_FOR
  for (int64_t r = 0; r < n; ++r) {
    double fr = g[r] - x[r];
    df[r] = fr - a->f_prev[r];
    dg[r] = g[r] - a->g_prev[r];
    a->f[r] = fr;
  }
  memcpy(a->f_prev, a->f, sizeof(double) * (size_t)n);
  memcpy(a->g_prev, g, sizeof(double) * (size_t)n);
  a->res_norm = nrm2(n, a->f);

  int st = OR_OK;
  if (i > m) st = or_qr_delete(s, a->variant, a->flags);
  if (st == OR_OK) st = or_qr_add(s, a->variant, a->flags, df);
  if (st != OR_OK) {
    a->status = st;
    return st;
  }
  or_qr_rhs(s, a->f, a->c);
  st = or_backsolve(s->k, s->cap, s->R, a->c, a->gamma);
  if (st != OR_OK) {
    a->status = st;
    return st;
  }
  OR_PARALLEL_FOR
  for (int64_t r = 0; r < n; ++r) {
    double acc = g[r];
    for (int j = 0; j < m_i; ++j) {
      int64_t col = (i - m_i + j) % m;
      acc -= a->gamma[j] * a->dG[col * s->ld + r];
    }
    x_next[r] = acc;
  }
  a->step_norm = sqrt(sqdist(n, x_next, x));
  a->m_i = m_i;
  a->i = i + 1;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* model problems (the fixed-point maps the workloads use)             */
/* ------------------------------------------------------------------ */

/* out = u - omega (A u + c u^3 - f), A the (2d+1)-point Dirichlet Laplacian
 * on an s^d grid with spacing h, x fastest:  (A u)_p = (2d u_p - sum of the
 * 2d neighbours) / h^2, neighbours outside the grid are 0. */
void or_G_stencil(int d, int64_t s, double h, double omega, double c,
                  const double *f, const double *u, double *out) {
  int64_t n = s;
  if (d >= 2) n *= s;
  if (d >= 3) n *= s;
  double ih2 = 1.0 / (h * h);
  OR_PARALLEL_FOR
  for (int64_t p = 0; p < n; ++p) {
    int64_t ix = p % s, iy = (p / s) % s, iz = p / (s * s);
    double nb = 0.0;
    if (ix > 0) nb += u[p - 1];
    if (ix < s - 1) nb += u[p + 1];
    if (d >= 2) {
      if (iy > 0) nb += u[p - s];
      if (iy < s - 1) nb += u[p + s];
    }
    if (d >= 3) {
      if (iz > 0) nb += u[p - s * s];
      if (iz < s - 1) nb += u[p + s * s];
    }
    double au = (2.0 * d * u[p] - nb) * ih2;
    out[p] = u[p] - omega * (au + c * u[p] * u[p] * u[p] - f[p]);
  }
}

/* y = A u for the same Laplacian (used by GMRES and residual checks). */
void or_laplacian(int d, int64_t s, double h, const double *u, double *y) {
  int64_t n = s;
  if (d >= 2) n *= s;
  if (d >= 3) n *= s;
  double ih2 = 1.0 / (h * h);
  OR_PARALLEL_FOR
  for (int64_t p = 0; p < n; ++p) {
    int64_t ix = p % s, iy = (p / s) % s, iz = p / (s * s);
    double nb = 0.0;
    if (ix > 0) nb += u[p - 1];
    if (ix < s - 1) nb += u[p + 1];
    if (d >= 2) {
      if (iy > 0) nb += u[p - s];
      if (iy < s - 1) nb += u[p + s];
    }
    if (d >= 3) {
      if (iz > 0) nb += u[p - s * s];
      if (iz < s - 1) nb += u[p + s * s];
    }
    y[p] = (2.0 * d * u[p] - nb) * ih2;
  }
}

/* ------------------------------------------------------------------ */
/* expectation-maximization of a normal mixture's means (Sec. 5.3)     */
/* ------------------------------------------------------------------ */

/* The EM update of the three means of a univariate mixture with known
 * proportions alpha and standard deviations sigma, from N samples x (Sec.
 * 5.3): with the current means mu (the first three entries of u),
 *   p_i(x_k) = alpha_i / (sqrt(2 pi) sigma_i) exp(-(x_k - mu_i)^2 / (2 sigma_i^2)),
 *   w_ik = p_i(x_k) / sum_j p_j(x_k),
 *   G(mu)_i = sum_k x_k w_ik / sum_k w_ik,
 * each sum over k compensated.  The result is written to every replica:
 * out[3 r + i] = G(mu)_i, r < n / 3. */
void or_G_em(int64_t n, const double *u, const double *x, int64_t N, const double *alpha,
             const double *sigma, double *out) {
  double num[3] = {0, 0, 0}, numc[3] = {0, 0, 0}, den[3] = {0, 0, 0}, denc[3] = {0, 0, 0};
  const double inv_sqrt_2pi = 0.39894228040143267793994605993438;
  for (int64_t k = 0; k < N; ++k) {
    double p[3], tot = 0.0;
    for (int i = 0; i < 3; ++i) {
      double d = x[k] - u[i];
      p[i] = alpha[i] * inv_sqrt_2pi / sigma[i] * exp(-(d * d) / (2.0 * sigma[i] * sigma[i]));
      tot += p[i];
    }
    for (int i = 0; i < 3; ++i) {
      double w = p[i] / tot;
      neumaier_add(&num[i], &numc[i], x[k] * w);
      neumaier_add(&den[i], &denc[i], w);
    }
  }
  double g[3];
  for (int i = 0; i < 3; ++i) g[i] = (num[i] + numc[i]) / (den[i] + denc[i]);
  OR_PARALLEL_FOR
  for (int64_t r = 0; r < n / 3; ++r)
    for (int i = 0; i < 3; ++i) out[3 * r + i] = g[i];
}

/* ------------------------------------------------------------------ */
/* GMRES (Saad and Schultz), used to pin AA through its equivalence    */
/* with GMRES for linear maps (Sec. 1).  Textbook form: Arnoldi with   */
/* modified Gram-Schmidt, Givens rotations on the Hessenberg matrix.   */
/* The operator is y = A x with A dense (n x n, column-major) when     */
/* A != NULL, else the Laplacian (d, s, h).  Writes the iterates       */
/* x_0 .. x_K into X (n x (K+1)); returns the number of iterates       */
/* written beyond x_0 (fewer than K on an exact breakdown).            */
/* ------------------------------------------------------------------ */

static void apply_op(int64_t n, const double *A, int d, int64_t s, double h,
                     const double *x, double *y) {
  if (A) {
    for (int64_t r = 0; r < n; ++r) y[r] = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t r = 0; r < n; ++r) y[r] += A[r + j * n] * x[j];
  } else {
    or_laplacian(d, s, h, x, y);
  }
}

int or_gmres(int64_t n, const double *A, int d, int64_t s, double h,
             const double *b, const double *x0, int K, double *X) {
  double *V = (double *)calloc((size_t)n * (size_t)(K + 1), sizeof(double));
  double *H = (double *)calloc((size_t)(K + 1) * (size_t)K, sizeof(double));
  double *cs = (double *)calloc((size_t)K, sizeof(double));
  double *sn = (double *)calloc((size_t)K, sizeof(double));
  double *e = (double *)calloc((size_t)(K + 1), sizeof(double));
  double *y = (double *)calloc((size_t)K + 1, sizeof(double));
  double *w = (double *)calloc((size_t)n, sizeof(double));
#define HM(i, j) H[(i) + (int64_t)(j) * (K + 1)]
  memcpy(X, x0, sizeof(double) * (size_t)n);
  apply_op(n, A, d, s, h, x0, w);
  for (int64_t r = 0; r < n; ++r) w[r] = b[r] - w[r];
  double beta = nrm2(n, w);
  int done = 0;
  if (beta > 0.0) {
    for (int64_t r = 0; r < n; ++r) V[r] = w[r] / beta;
    e[0] = beta;
    for (int j = 0; j < K; ++j) {
      apply_op(n, A, d, s, h, V + (int64_t)j * n, w);
      for (int i = 0; i <= j; ++i) {
        HM(i, j) = dot(n, V + (int64_t)i * n, w);
        axmy(n, HM(i, j), V + (int64_t)i * n, w);
      }
      double hnext = nrm2(n, w);
      HM(j + 1, j) = hnext;
      if (hnext > 0.0)
        for (int64_t r = 0; r < n; ++r) V[(int64_t)(j + 1) * n + r] = w[r] / hnext;
      /* previous rotations on column j, then a new one zeroing H_{j+1,j} */
      for (int i = 0; i < j; ++i) {
        double t0 = HM(i, j), t1 = HM(i + 1, j);
        HM(i, j) = cs[i] * t0 + sn[i] * t1;
        HM(i + 1, j) = -sn[i] * t0 + cs[i] * t1;
      }
      double a = HM(j, j), bb = HM(j + 1, j), rho = hypot(a, bb);
      cs[j] = rho > 0.0 ? a / rho : 1.0;
      sn[j] = rho > 0.0 ? bb / rho : 0.0;
      HM(j, j) = rho;
      HM(j + 1, j) = 0.0;
      e[j + 1] = -sn[j] * e[j];
      e[j] = cs[j] * e[j];
      /* x_{j+1} = x_0 + V_{:,0:j} y, with the (j+1) x (j+1) triangle */
      for (int i = j; i >= 0; --i) {
        double acc = e[i];
        for (int l = i + 1; l <= j; ++l) acc -= HM(i, l) * y[l];
        y[i] = acc / HM(i, i);
      }
      double *xj = X + (int64_t)(j + 1) * n;
      for (int64_t r = 0; r < n; ++r) {
        double acc = x0[r];
        for (int l = 0; l <= j; ++l) acc += V[(int64_t)l * n + r] * y[l];
        xj[r] = acc;
      }
      done = j + 1;
      if (hnext == 0.0) break; /* invariant Krylov space: x_{j+1} is exact */
    }
  }
#undef HM
  free(V); free(H); free(cs); free(sn); free(e); free(y); free(w);
  return done;
}
