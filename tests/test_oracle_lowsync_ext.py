"""Pins of the two QR-update forms Sec. 3 names besides Algs. 3-6:

* ICWY's T after QRDelete without a reduction (the T update of Sec. 3.2 read
  as a transformation of the old Gram matrix by the delete's rotations):
  its rows must equal the strict lower part of Q^T Q of the rotated basis,
  computed here directly with numpy, on bases that have lost orthogonality
  (so that T is far from the identity and every entry is checked for real);
* the delayed CGS-2 with the normalization lagged as well (Sec. 3.4): Q R
  equals the added columns after every add, and once the newest column has
  had its delayed reorthogonalization (the final step the lagged form needs)
  the basis is orthonormal to O(eps) -- what Sec. 3.4 reports for it -- and
  equals the positive-diagonal Householder QR on exact input.
"""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O

EPS = np.finfo(np.float64).eps


def graded_matrix(n, m, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (U * np.logspace(0, -np.log10(kappa), m)) @ V.T


def householder_qr_pos(A):
    Qh, Rh = np.linalg.qr(A, mode="reduced")
    sg = np.sign(np.diag(Rh))
    sg[sg == 0] = 1.0
    return Qh * sg, (Rh.T * sg).T


def gram_rows_ok(q, tol):
    """Rows 0..K-2 of T against strict-lower(Q^T Q) of the current basis (row
    K-1 is recomputed by the next QRAdd before any read, Alg. 4)."""
    K = q.k
    G = q.Qk().T @ q.Qk()
    T = q.Tk()
    err = 0.0
    for a in range(1, K - 1):
        err = max(err, np.abs(T[a, :a] - G[a, :a]).max())
    assert err <= tol, err
    return err


# ---------------------------------------------------------------- ICWY T transform

@pytest.mark.parametrize("kappa", [1e4, 1e8, 1e11])
@pytest.mark.parametrize("k", [2, 3, 6, 12])
def test_icwy_T_transform_equals_gram_of_rotated_basis(kappa, k):
    n = 300
    F = graded_matrix(n, k, kappa, seed=60 + k)
    q = O.QR(n, k, "icwy", O.ICWY_T_TRANSFORM)
    ref = O.QR(n, k, "icwy")
    for j in range(k):
        assert q.add(F[:, j]) == O.OK and ref.add(F[:, j]) == O.OK
    assert q.delete() == O.OK and ref.delete() == O.OK
    # the rotations are the same either way: Q and R bit for bit
    assert np.array_equal(q.Qk(), ref.Qk()) and np.array_equal(q.Rk(), ref.Rk())
    G = q.Qk().T @ q.Qk()
    tol = 50 * k * EPS
    if kappa >= 1e11 and k >= 6:
        # lost orthogonality: entries of T far above the tolerance, so a
        # misplaced or dropped one shows
        assert np.abs(np.tril(G, -1)).max() > 1e3 * tol
    gram_rows_ok(q, tol)
    # no reduction in the delete
    assert q.syncs[1] == 0 and ref.syncs[1] == 1


@pytest.mark.parametrize("m", [3, 5, 9])
def test_icwy_T_transform_through_window_recycling(m):
    """3m adds through a window of m (every add after the m-th follows a
    delete): Q R = F and T's rows stay the Gram of the current basis."""
    n = 257
    cols = graded_matrix(n, 3 * m, 1e6, seed=70 + m)
    q = O.QR(n, m, "icwy", O.ICWY_T_TRANSFORM)
    worst = 0.0
    for t in range(3 * m):
        if q.k == m:
            assert q.delete() == O.OK
            worst = max(worst, gram_rows_ok(q, 200 * m * EPS))
        assert q.add(cols[:, t]) == O.OK
        lo = max(0, t + 1 - m)
        Fw = cols[:, lo: t + 1]
        assert np.linalg.norm(Fw - q.Qk() @ q.Rk()) <= 10 * m * EPS * np.linalg.norm(Fw)
    assert q.syncs[1] == 0


def test_icwy_T_transform_aa_matches_recomputed_T():
    """AA with the transformed T against AA with the recomputed T: the same
    iterates to rounding (window m = 4 recycled from iteration 5)."""
    prob = W.nonlinear3d(s=10, seed=4)
    G = lambda u: O.G_stencil(prob, u)
    a, sa, _ = O.run_aa(G, np.zeros(prob.n), 4, "icwy", 25)
    b, sb, _ = O.run_aa(G, np.zeros(prob.n), 4, "icwy", 25, flags=O.ICWY_T_TRANSFORM)
    for i in range(1, 27):
        assert np.linalg.norm(a[i] - b[i]) <= 1e-11 * np.linalg.norm(a[i]), i
    assert sb.syncs[1] == 0 and sa.syncs[1] == 25 - 4


# ---------------------------------------------------------------- lagged DCGS-2

@pytest.mark.parametrize("kappa", [1e2, 1e5, 1e7])
def test_lagged_dcgs2_orthogonal_after_final_step(kappa):
    n, m = 400, 10
    F = graded_matrix(n, m, kappa, seed=81)
    q = O.QR(n, m, "dcgs2_lag")
    for j in range(m):
        assert q.add(F[:, j]) == O.OK
        assert np.linalg.norm(F[:, : j + 1] - q.Qk() @ q.Rk()) <= 10 * m * EPS * np.linalg.norm(F)
    Q = q.Qk()
    # every column but the newest has had its delayed reorthogonalization
    assert np.linalg.norm(np.eye(m - 1) - Q[:, : m - 1].T @ Q[:, : m - 1]) <= 50 * m * EPS
    assert q.flush() == O.OK
    Q, R = q.Qk(), q.Rk()
    assert np.linalg.norm(np.eye(m) - Q.T @ Q) <= 50 * m * EPS
    assert np.linalg.norm(F - Q @ R) <= 10 * m * EPS * np.linalg.norm(F)
    assert np.all(np.diag(R) > 0)
    _, Rh = householder_qr_pos(F)
    assert np.allclose(R, Rh, rtol=0, atol=100 * m * EPS * kappa * np.abs(Rh).max())


def test_lagged_dcgs2_orthogonality_beats_delayed_cgs2():
    """Sec. 3.4: the delayed CGS-2 of Alg. 6 loses orthogonality between
    O(eps) and O(eps) kappa^2; with its normalization lagged it stays O(eps)."""
    n, m = 400, 10
    F = graded_matrix(n, m, 1e7, seed=83)
    lag = O.QR(n, m, "dcgs2_lag")
    d = O.QR(n, m, "dcgs2")
    for j in range(m):
        lag.add(F[:, j])
        d.add(F[:, j])
    lag.flush()
    loss = lambda q: np.linalg.norm(np.eye(m) - q.Qk().T @ q.Qk())
    assert loss(lag) <= 50 * m * EPS < loss(d)


def test_lagged_dcgs2_one_reduction_per_add_and_flush_errors():
    n, m = 64, 6
    rng = np.random.default_rng(3)
    q = O.QR(n, m, "dcgs2_lag")
    for j in range(m):
        q.add(rng.standard_normal(n))
    assert q.syncs[0] == m
    q.delete()
    q.add(rng.standard_normal(n))
    assert q.syncs[0] == m + 1 and q.syncs[1] == 0
    assert q.flush() == O.OK and q.syncs[0] == m + 2
    assert O.QR(n, m, "cgs2").flush() == O.EINVAL


def test_lagged_dcgs2_breakdown_on_dependent_column():
    """A column already in the span: nu - ||r||^2 is rounding noise (here
    exactly zero or negative for a multiple of q_0 with n = 1)."""
    q = O.QR(1, 3, "dcgs2_lag")
    assert q.add(np.array([3.0])) == O.OK
    assert q.add(np.array([-2.0])) == O.EBREAKDOWN


def test_lagged_dcgs2_on_nonorthonormal_basis():
    """On a basis that has lost orthogonality (an MGS basis of a kappa = 1e12
    matrix, ~1e-4) the delayed corrections s are large, so each step shows:
    Q R = F still holds as an identity (R_{0:p-1,p} += R_pp s), the
    reorthogonalized previous column has unit norm (rho^2 = alpha - s^T s), and
    the new column is orthogonal to it (R_pk = (beta - s^T z) / rho)."""
    n, k = 150, 6
    F = graded_matrix(n, k, 1e12, seed=51)
    base = O.QR(n, k, "mgs")
    for j in range(k):
        base.add(F[:, j])
    Q0, R0 = base.Qk(), base.Rk()
    assert np.linalg.norm(np.eye(k) - Q0.T @ Q0) > 1e-6
    v = np.random.default_rng(52).standard_normal(n)
    q = O.QR(n, k + 1, "dcgs2_lag")
    q.Q[:, :k], q.R[:k, :k] = Q0, R0
    q.s.k = k
    assert q.add(v) == O.OK
    Fn = np.column_stack([Q0 @ R0, v])
    assert np.linalg.norm(Fn - q.Qk() @ q.Rk()) <= 100 * k * EPS * np.linalg.norm(Fn)
    qp, qk = q.Q[:, k - 1], q.Q[:, k]
    assert abs(np.linalg.norm(qp) - 1.0) <= 1e-12
    assert abs(qp @ qk) <= 1e-7
