"""Pins of the oracle's QR update (QRAdd Algs. 3-6, Givens QRDelete, Alg. 2).

Nothing here re-types the oracle's formulas.  The checks are what the paper
and linear algebra fix independently of any implementation:

* Q R equals the matrix whose columns were added (the factorization the
  window holds, Sec. 2.1), for every variant and after deletions;
* the loss of orthogonality ||I - Q^T Q|| stays within the bounds Sec. 2.2
  quotes (CGS-2 O(eps), MGS and ICWY O(eps) kappa);
* with an exactly orthonormal Q, every variant must return the new column of
  the unique positive-diagonal Householder QR of [Q v] (LAPACK via numpy);
* after QRDelete, R is the unique positive-diagonal R of the kept columns;
* the reduction counts equal the paper's stated counts (Sec. 3, Sec. 4.1);
* ICWY's solve with T = I + L reproduces MGS's coefficients, the identity
  (I + L) r = Q^T v that MGS satisfies by construction (Sec. 3.2).
"""
import os

import numpy as np
import pytest

import oracle as O

EPS = np.finfo(np.float64).eps
VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy"]
# with the delayed CGS-2 whose normalization is lagged too (Sec. 3.4)
VARIANTS_ALL = VARIANTS + ["dcgs2_lag"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graded_matrix(n, m, kappa, seed):
    """n x m matrix with singular values log-spaced in [1/kappa, 1]."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sv = np.logspace(0, -np.log10(kappa), m)
    return (U * sv) @ V.T


def householder_qr_pos(A):
    """Householder QR (LAPACK) with the signs fixed so that diag(R) > 0."""
    Qh, Rh = np.linalg.qr(A, mode="reduced")
    sg = np.sign(np.diag(Rh))
    sg[sg == 0] = 1.0
    return Qh * sg, (Rh.T * sg).T


def fill(variant, F, flags=0):
    n, m = F.shape
    q = O.QR(n, m, variant, flags)
    for j in range(m):
        assert q.add(F[:, j]) == O.OK
    return q


@pytest.mark.parametrize("variant", VARIANTS_ALL)
@pytest.mark.parametrize("kappa", [1e1, 1e4, 1e7])
def test_qr_equals_F_after_adds(variant, kappa):
    F = graded_matrix(300, 8, kappa, seed=11)
    q = fill(variant, F)
    Q, R = q.Qk(), q.Rk()
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.all(np.diag(R) > 0)
    err = np.linalg.norm(F - Q @ R) / np.linalg.norm(F)
    assert err <= 10 * 8 * EPS, err


@pytest.mark.parametrize("variant", VARIANTS_ALL)
def test_qr_equals_F_through_window_recycling(variant):
    """Add 3m columns through a window of m: delete the oldest when full."""
    n, m = 257, 5
    rng = np.random.default_rng(5)
    cols = rng.standard_normal((n, 3 * m))
    q = O.QR(n, m, variant)
    for t in range(3 * m):
        if q.k == m:
            assert q.delete() == O.OK
        assert q.add(cols[:, t]) == O.OK
        lo = max(0, t + 1 - m)
        F = cols[:, lo: t + 1]
        Q, R = q.Qk(), q.Rk()
        assert np.linalg.norm(F - Q @ R) / np.linalg.norm(F) <= 10 * m * EPS
        assert np.linalg.norm(np.eye(q.k) - Q.T @ Q) <= 1e-13


@pytest.mark.parametrize("kappa", [1e2, 1e5, 1e8])
def test_loss_of_orthogonality_bounds(kappa):
    """Sec. 2.2: CGS-2 O(eps); MGS and ICWY O(eps) kappa; DCGS-2 in between
    O(eps) and O(eps) kappa^2."""
    n, m = 400, 10
    F = graded_matrix(n, m, kappa, seed=21)
    loss = {}
    for v in VARIANTS:
        Q = fill(v, F).Qk()
        loss[v] = np.linalg.norm(np.eye(m) - Q.T @ Q)
    assert loss["cgs2"] <= 50 * m * EPS
    assert loss["mgs"] <= 50 * m * EPS * kappa
    assert loss["icwy"] <= 50 * m * EPS * kappa
    assert loss["dcgs2"] <= 50 * m * EPS * kappa ** 2


def test_mgs_loss_grows_with_kappa():
    """MGS loses orthogonality in proportion to kappa (Bjorck) while CGS-2
    does not, so the bounds above are not vacuous."""
    n, m = 400, 10

    def loss(variant, kappa):
        Q = fill(variant, graded_matrix(n, m, kappa, 3)).Qk()
        return np.linalg.norm(np.eye(m) - Q.T @ Q)

    assert loss("mgs", 1e10) > 100 * loss("mgs", 1e2)
    assert loss("cgs2", 1e10) <= 50 * m * EPS


@pytest.mark.parametrize("variant", VARIANTS_ALL)
@pytest.mark.parametrize("k", [0, 1, 2, 3, 5, 9])
def test_new_column_matches_householder(variant, k):
    """Exactly orthonormal Q and Gaussian v: every variant returns the last
    column of the positive-diagonal Householder QR of [Q v]."""
    n = 120
    rng = np.random.default_rng(100 + k)
    A = rng.standard_normal((n, k + 1))
    Qh, Rh = householder_qr_pos(A)
    q = O.QR(n, k + 1, variant)
    q.Q[:, :k] = Qh[:, :k]
    q.R[:k, :k] = Rh[:k, :k]
    q.T[:k, :k] = np.eye(k)
    q.s.k = k
    assert q.add(A[:, k]) == O.OK
    assert np.allclose(q.Q[:, k], Qh[:, k], rtol=0, atol=1e-13)
    assert np.allclose(q.R[: k + 1, k], Rh[:, k], rtol=0, atol=1e-13 * np.abs(Rh).max())


@pytest.mark.parametrize("variant", VARIANTS_ALL)
@pytest.mark.parametrize("m", [2, 3, 6])
def test_delete_gives_unique_R_of_kept_columns(variant, m):
    n = 90
    F = graded_matrix(n, m, 1e3, seed=7 + m)
    q = fill(variant, F)
    assert q.delete() == O.OK
    assert q.k == m - 1
    Q, R = q.Qk(), q.Rk()
    _, Rh = householder_qr_pos(F[:, 1:])
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(R, Rh, rtol=0, atol=10 * m * EPS * 1e3 * np.abs(Rh).max())
    assert np.linalg.norm(F[:, 1:] - Q @ R) / np.linalg.norm(F) <= 10 * m * EPS
    if variant == "icwy":
        # A5 reading: T is refreshed to I + strict-lower(Q^T Q) of the new Q
        G = Q.T @ Q
        assert np.allclose(q.Tk(), np.eye(m - 1) + np.tril(G, -1), rtol=0, atol=1e-15)


def test_delete_single_column_and_empty_window_errors():
    q = O.QR(10, 2, "mgs")
    assert q.delete() == O.ESTATE
    q.add(np.arange(10.0) + 1)
    assert q.delete() == O.OK and q.k == 0
    q.add(np.ones(10))
    q.add(np.arange(10.0))
    assert q.add(np.ones(10) * 3) == O.ESTATE  # window full


@pytest.mark.parametrize("variant", VARIANTS_ALL)
def test_breakdown_is_reported(variant):
    q = O.QR(16, 3, variant)
    assert q.add(np.zeros(16)) == O.EBREAKDOWN
    q2 = O.QR(16, 3, variant)
    v = np.ones(16)
    v[3] = np.nan
    assert q2.add(v) == O.EBREAKDOWN


def _golden_syncs():
    rows = {}
    for line in open(os.path.join(GOLDEN, "sync_counts.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        name, a, b, c, d, rec, dele = line
        rows[name] = (int(a), int(b), int(c), int(d), rec, int(dele))
    return rows


@pytest.mark.parametrize("variant", VARIANTS_ALL)
@pytest.mark.parametrize("m", [1, 2, 3, 4, 7, 12])
def test_sync_counts_match_paper(variant, m):
    a, b, c, d, rec, dele = _golden_syncs()[variant]
    n = 64
    rng = np.random.default_rng(m)
    q = O.QR(n, m, variant)
    for j in range(m):
        q.add(rng.standard_normal(n))
    assert q.syncs[0] == (a * m * m + b * m + c) // d
    # one recycle iteration: delete, then add against m - 1 columns
    before = q.syncs
    q.delete()
    q.add(rng.standard_normal(n))
    after = q.syncs
    expect_add = m if rec == "m" else (int(rec) if m > 1 else 1)
    assert after[0] - before[0] == expect_add
    assert after[1] - before[1] == (dele if m > 1 else 0)
    q.rhs(rng.standard_normal(n))
    assert q.syncs[2] == 1 and q.syncs[0] == after[0]


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10, 1e12])
def test_icwy_equals_mgs_coefficients(kappa):
    """(I + L) r = Q^T v holds for MGS's coefficients, so ICWY (which solves
    with T = I + L, Alg. 4) must reproduce MGS's R column on the same Q."""
    n, k = 200, 7
    F = graded_matrix(n, k, kappa, seed=31)
    base = fill("mgs", F)
    Q = base.Qk()
    v = np.random.default_rng(32).standard_normal(n)
    L = np.tril(Q.T @ Q, -1)
    cols = {}
    for variant in ("mgs", "icwy"):
        q = O.QR(n, k + 1, variant)
        q.Q[:, :k] = Q
        q.R[:k, :k] = base.Rk()
        # T's rows 0..k-2 as ICWY would have built them; row k-1 is recomputed
        q.T[:k, :k] = np.eye(k) + L
        q.s.k = k
        assert q.add(v) == O.OK
        cols[variant] = q.R[:k, k].copy()
    r = cols["mgs"]
    assert np.linalg.norm((np.eye(k) + L) @ r - Q.T @ v) <= 100 * EPS * np.linalg.norm(v) * k
    # no kappa slack: both routes evaluate the same identity, while at
    # kappa = 1e10 the entries of L are ~1e-7, so any slip in T shows
    assert np.allclose(cols["icwy"], r, rtol=0, atol=100 * k * EPS * np.linalg.norm(v))


@pytest.mark.parametrize("variant", VARIANTS_ALL)
def test_qr_equals_F_with_nonorthonormal_basis(variant):
    """Each variant's update satisfies Q R = F as an algebraic identity, even
    when the stored basis has lost orthogonality (here ~1e-4, an MGS basis of
    a kappa = 1e12 matrix).  Corrections that are O(eps) for an orthonormal
    basis (CGS-2's z, DCGS-2's s) are then large, so dropping one shows."""
    n, k = 150, 6
    F = graded_matrix(n, k, 1e12, seed=51)
    base = fill("mgs", F)
    Q0, R0 = base.Qk(), base.Rk()
    assert np.linalg.norm(np.eye(k) - Q0.T @ Q0) > 1e-6
    v = np.random.default_rng(52).standard_normal(n)
    q = O.QR(n, k + 1, variant)
    q.Q[:, :k] = Q0
    q.R[:k, :k] = R0
    q.T[:k, :k] = np.eye(k) + np.tril(Q0.T @ Q0, -1)
    q.s.k = k
    assert q.add(v) == O.OK
    Fn = np.column_stack([Q0 @ R0, v])
    err = np.linalg.norm(Fn - q.Qk() @ q.Rk()) / np.linalg.norm(Fn)
    assert err <= 100 * k * EPS, err


def test_dcgs2_literal_reading_breaks_qr_equals_F():
    """Alg. 6 read literally (R += s) keeps Q R = F only if R_{k-1,k-1} = 1;
    the default reading (R += R_{k-1,k-1} s) keeps it always."""
    n, m = 200, 6
    F = graded_matrix(n, m, 1e6, seed=41) * 37.0
    q_def = fill("dcgs2", F)
    q_lit = fill("dcgs2", F, flags=O.DCGS2_LITERAL)
    e_def = np.linalg.norm(F - q_def.Qk() @ q_def.Rk()) / np.linalg.norm(F)
    e_lit = np.linalg.norm(F - q_lit.Qk() @ q_lit.Rk()) / np.linalg.norm(F)
    assert e_def <= 10 * m * EPS
    assert e_lit > 1e3 * e_def


def test_dcgs2_reorthogonalization_guard():
    """m_i > 3 guard: the third column (m_i = 3) is not reorthogonalized, the
    fourth (m_i = 4) is (2 reductions either way)."""
    n = 150
    F = graded_matrix(n, 5, 1e6, seed=43)
    q = O.QR(n, 5, "dcgs2")
    q.add(F[:, 0]); q.add(F[:, 1])
    q1 = q.Q[:, 1].copy()
    q.add(F[:, 2])
    assert np.array_equal(q.Q[:, 1], q1)       # m_i = 3: q_1 untouched
    q2 = q.Q[:, 2].copy()
    q.add(F[:, 3])
    assert not np.array_equal(q.Q[:, 2], q2)   # m_i = 4: q_2 reorthogonalized
    g = O.QR(n, 5, "dcgs2", flags=O.DCGS2_GUARD_GE3)
    g.add(F[:, 0]); g.add(F[:, 1])
    q1 = g.Q[:, 1].copy()
    g.add(F[:, 2])
    assert not np.array_equal(g.Q[:, 1], q1)


@pytest.mark.parametrize("variant", VARIANTS_ALL)
def test_breakdown_on_a_repeated_column_only(variant):
    """Reading A10: a column numerically in the span of the window (R_kk at
    most 64 eps times its column norm) is a breakdown; a column 1e-9 away from
    the span is not.  The lagged DCGS-2 takes the new column's norm from
    Pythagoras, which resolves a distance above ~sqrt(eps) only (reading
    A19): 1e-6 there."""
    rng = np.random.default_rng(61)
    n = 200
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    q = O.QR(n, 3, variant)
    assert q.add(a) == O.OK
    assert q.add(a.copy()) == O.EBREAKDOWN
    q2 = O.QR(n, 3, variant)
    assert q2.add(a) == O.OK
    d = 1e-6 if variant == "dcgs2_lag" else 1e-9
    assert q2.add(a + d * b) == O.OK
    R = q2.Rk()
    assert R[1, 1] / np.linalg.norm(R[:, 1]) > d / 10
