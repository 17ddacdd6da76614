"""Pins of the oracle's Anderson-acceleration loop (Alg. 1 with Alg. 2).

* gamma against the exact least-squares solution of the FP64 data, computed in
  rational arithmetic (``fractions``) from the normal equations, on tiny n;
* gamma against the "definition" route: Householder QR of the explicit F_i;
* for linear G, AA without truncation equals GMRES applied to the same system
  (Sec. 1, via Walker and Ni): x^AA_{k+1} = G(x^GMRES_k); GMRES itself is
  pinned against a brute-force minimal-residual solve over the Krylov basis;
* n = 1, m = 1 reduces AA to the secant method (closed form);
* linear G with m >= n terminates in at most n + 1 iterations (GMRES finite
  termination);
* the window bookkeeping: x_{i+1} = G(x_i) - sum_j gamma_j Delta g_{i-m_i+j}
  with the columns of the ring in window order, checked against an explicit
  history of all iterates.
"""
from fractions import Fraction

import numpy as np
import pytest

import aa_workloads as W
import oracle as O

EPS = np.finfo(np.float64).eps
VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy", "dcgs2_lag"]


def spd(n, seed, shift=0.5):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return M @ M.T / n + shift * np.eye(n)


def linear_map(A, b):
    om = 0.9 / np.linalg.eigvalsh(A).max()
    return (lambda x: x - om * (A @ x - b)), om


def exact_lsq(F, f):
    """argmin ||f - F g|| exactly for the given FP64 data (normal equations in
    rational arithmetic, Gauss-Jordan elimination)."""
    n, k = F.shape
    Fr = [[Fraction(float(F[r, j])) for j in range(k)] for r in range(n)]
    fr = [Fraction(float(f[r])) for r in range(n)]
    M = [[sum(Fr[r][a] * Fr[r][b] for r in range(n)) for b in range(k)]
         + [sum(Fr[r][a] * fr[r] for r in range(n))] for a in range(k)]
    for c in range(k):
        piv = next(r for r in range(c, k) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(k):
            if r != c and M[r][c] != 0:
                t = M[r][c] / M[c][c]
                M[r] = [M[r][j] - t * M[c][j] for j in range(k + 1)]
    return np.array([float(M[a][k] / M[a][a]) for a in range(k)])


@pytest.mark.parametrize("variant", VARIANTS)
def test_gamma_matches_exact_rational_lsq(variant):
    n, m = 7, 3
    A = spd(n, 1)
    b = np.random.default_rng(2).standard_normal(n)
    G, _ = linear_map(A, b)
    st = O.AA(n, m, variant)
    x = np.zeros(n)
    for it in range(6):
        g = G(x)
        x_new = st.step(x, g)
        if st.i >= 2:
            F, f = st.F(), st.f.copy()
            gam = st.gamma_k()
            exact = exact_lsq(F, f)
            kap = np.linalg.cond(F)
            assert np.allclose(gam, exact, rtol=0, atol=10 * kap * EPS * np.abs(exact).max() + 1e-300)
            # the LSP residual is orthogonal to range(F)
            res = f - F @ gam
            assert np.linalg.norm(F.T @ res) <= 10 * kap * EPS * np.linalg.norm(F) * np.linalg.norm(f)
        x = x_new


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("m", [1, 2, 4])
def test_step_against_definition_and_history(variant, m):
    """Per-variant step vs the definition: gamma from Householder LSP of the
    explicit F_i (window order), x_{i+1} from an explicit list of G(x_k)."""
    prob = W.nonlinear3d(s=6, seed=9)
    n = prob.n
    st = O.AA(n, m, variant)
    x = np.zeros(n)
    xs, gs = [], []
    for i in range(12):
        g = O.G_stencil(prob, x)
        xs.append(x.copy()); gs.append(g.copy())
        x_next = st.step(x, g)
        if i == 0:
            assert np.array_equal(x_next, g)
        else:
            mi = min(m, i)
            fs = [gs[j] - xs[j] for j in range(i + 1)]
            F = np.stack([fs[j + 1] - fs[j] for j in range(i - mi, i)], 1)
            Gm = np.stack([gs[j + 1] - gs[j] for j in range(i - mi, i)], 1)
            assert st.m_i == mi
            assert np.array_equal(st.F(), F)
            gam = O.lsp_definition(F, fs[i])
            kap = np.linalg.cond(F)
            assert np.allclose(st.gamma_k(), gam, rtol=0,
                               atol=100 * kap * EPS * max(1.0, np.abs(gam).max()))
            ref = gs[i] - Gm @ st.gamma_k()
            assert np.allclose(x_next, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
            assert np.linalg.norm(F - st.Qk() @ st.Rk()) <= 10 * mi * EPS * np.linalg.norm(F)
        x = x_next


def test_gmres_matches_bruteforce_krylov():
    n = 25
    A = spd(n, 3)
    b = np.random.default_rng(4).standard_normal(n)
    x0 = np.random.default_rng(5).standard_normal(n) * 0.1
    X = O.gmres(b, x0, 8, A=A)
    r0 = b - A @ x0
    for k in range(1, 9):
        Kr = np.stack([np.linalg.matrix_power(A, j) @ r0 for j in range(k)], 1)
        y = np.linalg.lstsq(A @ Kr, r0, rcond=None)[0]
        xk = x0 + Kr @ y
        assert np.linalg.norm(X[:, k] - xk) <= 1e-10 * np.linalg.norm(xk)


def test_gmres_stencil_operator_matches_dense():
    s = 12
    prob = W.poisson1d(n=s, seed=3)
    A = np.diag(2.0 * np.ones(s)) - np.diag(np.ones(s - 1), 1) - np.diag(np.ones(s - 1), -1)
    A /= prob.h ** 2
    X1 = O.gmres(prob.f, np.zeros(s), 6, A=A)
    X2 = O.gmres(prob.f, np.zeros(s), 6, d=1, s=s, h=prob.h)
    assert np.allclose(X1, X2, rtol=0, atol=1e-12 * np.abs(X1).max())


@pytest.mark.parametrize("variant", VARIANTS)
def test_aa_equals_gmres_dense(variant):
    n = 30
    A = spd(n, 1)
    b = np.random.default_rng(1).standard_normal(n)
    G, _ = linear_map(A, b)
    x0 = np.zeros(n)
    K = 12
    X = O.gmres(b, x0, K, A=A)
    xs, _, _ = O.run_aa(G, x0, m=K + 5, variant=variant, iters=K)
    for k in range(K):
        ref = G(X[:, k])
        assert np.linalg.norm(xs[k + 1] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("variant", VARIANTS)
def test_aa_equals_gmres_poisson1d_n4096(variant):
    """The 1D Poisson workload (n = 4096, kappa ~ 6.8e6) with m = 25."""
    prob = W.poisson1d()
    n = prob.n
    G = lambda x: O.G_stencil(prob, x)
    x0 = np.zeros(n)
    K = 20
    X = O.gmres(prob.f, x0, K, d=1, s=n, h=prob.h)
    xs, _, _ = O.run_aa(G, x0, m=25, variant=variant, iters=K)
    for k in range(K):
        ref = G(X[:, k])
        assert np.linalg.norm(xs[k + 1] - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("variant", VARIANTS)
def test_secant_method_n1_m1(variant):
    """n = 1, m = 1: x_{i+1} = x_i - f_i (x_i - x_{i-1}) / (f_i - f_{i-1})."""
    G = lambda x: np.cos(x)            # fixed point of cos, f(x) = cos x - x
    st = O.AA(1, 1, variant)
    x_prev = np.array([0.3])
    x = st.step(x_prev, G(x_prev))
    for _ in range(5):
        f_i, f_prev = G(x) - x, G(x_prev) - x_prev
        secant = x - f_i * (x - x_prev) / (f_i - f_prev)
        x_next = st.step(x, G(x))
        assert abs(x_next[0] - secant[0]) <= 4 * EPS * max(1.0, abs(secant[0]))
        if abs(f_i[0]) < 1e-15:
            break
        x_prev, x = x, x_next


@pytest.mark.parametrize("variant", VARIANTS)
def test_finite_termination_linear(variant):
    """Linear G, n = 8, m >= n: converged after at most n + 1 iterations."""
    n = 8
    A = spd(n, 7, shift=1.0)
    b = np.random.default_rng(8).standard_normal(n)
    G, _ = linear_map(A, b)
    x = np.zeros(n)
    st = O.AA(n, n + 2, variant)
    for _ in range(n + 1):
        x = st.step(x, G(x))
    kap = np.linalg.cond(A)
    assert np.linalg.norm(A @ x - b) <= 1e3 * kap * EPS * np.linalg.norm(b)


@pytest.mark.parametrize("variant", VARIANTS)
def test_m1_closed_form(variant):
    """m = 1: gamma = Delta f^T f_i / ||Delta f||^2."""
    prob = W.nonlinear3d(s=5, seed=4)
    st = O.AA(prob.n, 1, variant)
    x = np.zeros(prob.n)
    f_prev = None
    for i in range(6):
        g = O.G_stencil(prob, x)
        f = g - x
        x_new = st.step(x, g)
        if i >= 1:
            df = f - f_prev
            assert abs(st.gamma_k()[0] - df @ f / (df @ df)) <= 1e-13 * abs(df @ f / (df @ df))
        f_prev, x = f, x_new


@pytest.mark.parametrize("variant", VARIANTS)
def test_nonlinear_convergence_small(variant):
    """AA drives the small 3D nonlinear problem to the 1e-8 residual tolerance."""
    prob = W.nonlinear3d(s=8, seed=2)
    G = lambda u: O.G_stencil(prob, u)
    xs, st, res = O.run_aa(G, np.zeros(prob.n), m=10, variant=variant, iters=400, tol=1e-8)
    assert res[-1] <= 1e-8 * st.res0_norm
    assert len(res) < 400


def test_variants_agree_on_well_conditioned_run():
    prob = W.nonlinear3d(s=6, seed=5)
    G = lambda u: O.G_stencil(prob, u)
    runs = {v: O.run_aa(G, np.zeros(prob.n), m=4, variant=v, iters=15)[0] for v in VARIANTS}
    for v in VARIANTS:
        for i, (a, b) in enumerate(zip(runs[v], runs["mgs"])):
            assert np.linalg.norm(a - b) <= 1e-9 * max(1.0, np.linalg.norm(b)), (v, i)
