"""Pins of the oracle's 2D test problems (Sec. 5.1 heat equation with a
nonlinear term, Sec. 5.2 Bratu) and of the PCG + geometric multigrid solve
inside their maps, each against something other than the oracle's own code:

* the operator against its eigendecomposition by the discrete sine transform
  (scipy's DST-I), and the PCG solution against the DST's exact solve;
* the coarse operators against the 1D Galerkin products R A P built from
  dense interpolation matrices written out from the hat functions;
* interpolation and full weighting against brute-force loops over the
  stencils, and interpolation reproducing a bilinear function exactly;
* a Gauss-Seidel half-sweep zeroing the residual at the swept colour;
* the V-cycle a symmetric positive definite operator, contracting the error
  by a mesh-independent factor;
* PCG with n iterations against a dense solve (finite termination);
* the manufactured solution of Sec. 5.1 reached at second order in h;
* the fixed points of both problems satisfying the discrete equations,
  written out point by point on a small grid;
* the iteration counts the paper reports as loose checks."""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import aa_workloads as W
import oracle as O
from oracle import pde2d as P


def rng(seed=0):
    return np.random.default_rng(seed)


def dst_eigs(N, h):
    k = np.arange(1, N + 1)
    lam1 = (4.0 / (h * h)) * np.sin(k * np.pi / (2 * (N + 1))) ** 2
    return lam1[:, None] + lam1[None, :]


def dst_apply(U, h, inverse=False):
    lam = dst_eigs(U.shape[0], h)
    c = sfft.dstn(U, type=1, norm="ortho")
    c = c / lam if inverse else c * lam
    return sfft.idstn(c, type=1, norm="ortho")


@pytest.mark.parametrize("N", [7, 16, 33])
def test_operator_matches_sine_transform(N):
    h = 1.0 / (N + 1)
    U = rng(N).standard_normal((N, N))
    assert np.allclose(P.apply_A(U, h), dst_apply(U, h), rtol=0, atol=1e-9 / (h * h))


def interp_matrix(N):
    """Linear interpolation from coarse points X_I = (2I + 2) h (I < N/2) to
    fine points x_i = (i + 1) h by the hat functions of the coarse grid (the
    boundary x = 0 carries zero)."""
    h = 1.0 / (N + 1)
    Nc = N // 2
    X = (2 * np.arange(Nc) + 2) * h
    M = np.zeros((N, Nc))
    for i in range(N):
        x = (i + 1) * h
        for I in range(Nc):
            M[i, I] = max(0.0, 1.0 - abs(x - X[I]) / (2 * h))
    return M


@pytest.mark.parametrize("N,levels", [(16, 3), (24, 3), (64, 5)])
def test_coarse_operators_are_the_1d_galerkin_products(N, levels):
    h = 1.0 / (N + 1)
    A1 = (2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)) / (h * h)
    n, H = N, h
    for lev in range(1, levels + 1):
        Pm = interp_matrix(n)  # positions relative to the spacing: any level
        A1 = (Pm.T / 2.0) @ A1 @ Pm
        n //= 2
        H *= 2
        U = rng(lev).standard_normal((n, n))
        ref = A1 @ U + U @ A1.T  # Kronecker sum acting on U[j, i]
        assert np.allclose(P.apply_A(U, H, lev), ref, rtol=1e-12, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("N", [8, 30])
def test_interpolation_brute_force_and_bilinear_exactness(N):
    h = 1.0 / (N + 1)
    Nc = N // 2
    Ec = rng(1).standard_normal((Nc, Nc))
    M = interp_matrix(N)
    assert np.allclose(P.prolong(Ec), M @ Ec @ M.T, rtol=0, atol=1e-13)
    # a bilinear function vanishing on the two boundaries x = 0 and y = 0
    g = lambda x, y: 2.5 * x * y
    Xc = (2 * np.arange(Nc) + 2) * h
    xf = (np.arange(N) + 1) * h
    Gc = np.array([[g(Xc[I], Xc[J]) for I in range(Nc)] for J in range(Nc)])
    Gf = np.array([[g(xf[i], xf[j]) for i in range(N)] for j in range(N)])
    assert np.allclose(P.prolong(Gc), Gf, rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [8, 22])
def test_full_weighting_brute_force(N):
    R = rng(2).standard_normal((N, N))
    Nc = N // 2
    w = {(0, 0): 4, (1, 0): 2, (-1, 0): 2, (0, 1): 2, (0, -1): 2,
         (1, 1): 1, (1, -1): 1, (-1, 1): 1, (-1, -1): 1}
    ref = np.zeros((Nc, Nc))
    for J in range(Nc):
        for I in range(Nc):
            s = 0.0
            for (dj, di), wt in w.items():
                j, i = 2 * J + 1 + dj, 2 * I + 1 + di
                if 0 <= j < N and 0 <= i < N:
                    s += wt * R[j, i]
            ref[J, I] = s / 16.0
    assert np.allclose(P.restrict(R), ref, rtol=0, atol=1e-15)
    # adjoint: <R r, e> = <r, P e> / 4
    Ec = rng(3).standard_normal((Nc, Nc))
    assert math.isclose(np.vdot(P.restrict(R), Ec), np.vdot(R, P.prolong(Ec)) / 4.0,
                        rel_tol=1e-13)


@pytest.mark.parametrize("level", [0, 2])
def test_gauss_seidel_half_sweep_zeroes_its_colour(level):
    N, h = 12, 0.1
    Rhs = rng(4).standard_normal((N, N))
    E = rng(5).standard_normal((N, N))
    for colour in (P.RED, P.BLACK):
        P.gs_colour(E, Rhs, h, colour, level)
        res = Rhs - P.apply_A(E, h, level)
        mask = P.colour_mask(N, colour)
        assert np.abs(res[mask]).max() <= 1e-10
        assert np.abs(res[~mask]).max() > 1e-6  # the other colour is not solved


def dense_B(N):
    h = 1.0 / (N + 1)
    n = N * N
    B = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        B[:, c] = P.vcycle(e.reshape(N, N), h).reshape(-1)
    return B, h


@pytest.mark.parametrize("N", [16, 12])
def test_vcycle_is_symmetric_positive_definite(N):
    B, _ = dense_B(N)
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0


def dense_A(N):
    h = 1.0 / (N + 1)
    n = N * N
    A = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = P.apply_A(e.reshape(N, N), h).reshape(-1)
    return A


@pytest.mark.parametrize("N", [8, 16, 32])
def test_vcycle_contracts_the_error_independently_of_h(N):
    """The V-cycle's error propagator I - B A has spectral radius well below
    1, and the same on every grid size (multigrid's defining property)."""
    B, _ = dense_B(N)
    A = dense_A(N)
    rho = np.abs(np.linalg.eigvals(np.eye(N * N) - B @ A)).max()
    assert rho < 0.3


def test_pcg_solution_matches_sine_transform_solve():
    N = 64
    h = 1.0 / (N + 1)
    rhs = rng(6).standard_normal((N, N))
    x, its, ok = P.pcg(rhs, h, 1e-13, 100)
    ref = dst_apply(rhs, h, inverse=True)
    assert ok and its <= 16
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    # the stopping test is the relative residual
    r = rhs - P.apply_A(x, h)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(rhs)


def test_pcg_terminates_in_n_steps_on_a_dense_check():
    N = 6
    h = 1.0 / (N + 1)
    rhs = rng(7).standard_normal((N, N))
    x, its, _ = P.pcg(rhs, h, 0.0, 1000, fixed_iters=12)
    ref = np.linalg.solve(dense_A(N), rhs.reshape(-1)).reshape(N, N)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("N", [32, 128])
def test_pcg_iterations_do_not_grow_with_the_grid(N):
    h = 1.0 / (N + 1)
    _, its, ok = P.pcg(rng(8).standard_normal((N, N)), h, 1e-10, 100)
    assert ok and 8 <= its <= 11


def solve(prob, variant="mgs", iters=80):
    Gf = lambda u: P.G(prob.problem, u, prob.N, prob.b, prob.lam)
    xs, st, res = O.run_aa(Gf, prob.u0(), prob.m, variant, iters=iters, tol=prob.tol)
    return xs[-1], len(res) - 1, st


@pytest.mark.parametrize("term", [W.PDE_HEAT_NL1, W.PDE_HEAT_NL2])
def test_manufactured_solution_second_order(term):
    """The discrete solution of Sec. 5.1 approaches sin^2(pi x) sin^2(pi y) at
    second order: doubling N (h ~ 1/(N+1)) divides the max error by ~((2N+1)
    /(N+1))^2.  A wrong sign or term in the source, the operator or c(u)
    leaves an O(1) error instead."""
    errs = []
    Ns = [16, 32, 64]
    for N in Ns:
        prob = W.heat2d(N, term)
        u, _, _ = solve(prob)
        errs.append(np.abs(u - W.heat_exact(N)).max())
    for a in range(2):
        ratio = errs[a] / errs[a + 1]
        expect = ((Ns[a + 1] + 1) / (Ns[a] + 1)) ** 2
        assert 0.85 * expect < ratio < 1.15 * expect, (errs, ratio, expect)
    assert errs[-1] < 2e-3


def equations_by_loops(prob, u):
    """L_h u + c(u) - f (heat) or L_h u + lam e^u (Bratu), written point by
    point with math.exp."""
    N, h = prob.N, prob.h
    U = u.reshape(N, N)
    out = np.zeros((N, N))
    for j in range(N):
        for i in range(N):
            nb = 0.0
            for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                jj, ii = j + dj, i + di
                if 0 <= jj < N and 0 <= ii < N:
                    nb += U[jj, ii]
            lap = (nb - 4.0 * U[j, i]) / (h * h)
            v = U[j, i]
            if prob.problem == W.PDE_HEAT_NL1:
                cv = v + v * math.exp(v) + v * math.exp(-v) + (v - math.exp(v)) ** 2
                out[j, i] = lap + cv - prob.b[j * N + i]
            elif prob.problem == W.PDE_HEAT_NL2:
                out[j, i] = lap + 100.0 * (v - v * v) - prob.b[j * N + i]
            else:
                out[j, i] = lap + prob.lam * math.exp(v)
    return out.reshape(-1)


@pytest.mark.parametrize("make", [lambda: W.heat2d(16, W.PDE_HEAT_NL1),
                                  lambda: W.heat2d(16, W.PDE_HEAT_NL2),
                                  lambda: W.bratu2d(16)])
def test_fixed_point_satisfies_the_discrete_equations(make):
    prob = make()
    u, its, _ = solve(prob)
    eq = equations_by_loops(prob, u)
    scale = 4.0 / prob.h ** 2 * np.abs(u).max()
    assert np.abs(eq).max() <= 1e-8 * scale
    assert np.allclose(eq, P.residual(prob.problem, u, prob.N, prob.b, prob.lam),
                       rtol=0, atol=1e-9 * scale)


def test_bratu_solution_has_the_squares_symmetry():
    prob = W.bratu2d(24)
    u, _, _ = solve(prob)
    U = u.reshape(24, 24)
    s = np.abs(U).max()
    assert np.abs(U - U.T).max() <= 1e-8 * s
    assert np.abs(U - U[::-1, :]).max() <= 1e-8 * s
    assert np.abs(U - U[:, ::-1]).max() <= 1e-8 * s
    assert U.min() > 0  # lam e^u > 0 pushes u up everywhere


@pytest.mark.parametrize("prob_id,m,lo,hi", [
    (W.PDE_HEAT_NL1, 5, 5, 14),     # the paper: 11 iterations for every variant
    (W.PDE_HEAT_NL2, 10, 27, 50),   # the paper: 27 to 42, DCGS-2 more
    (W.PDE_BRATU, 30, 5, 29),       # the paper: fewer than 30
])
def test_iteration_counts_near_the_papers(prob_id, m, lo, hi):
    N = 64
    prob = W.bratu2d(N) if prob_id == W.PDE_BRATU else W.heat2d(N, prob_id)
    assert prob.m == m
    for v in ("mgs", "icwy"):
        _, its, _ = solve(prob, v, iters=120)
        assert lo <= its <= hi, (v, its)


# --------------------------------------------------------------------------
# planted mistakes: each must make one of the pins above fail
# --------------------------------------------------------------------------

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_mutant_coarse_boundary_at_the_rediscretized_distance(monkeypatch):
    monkeypatch.setattr(P, "diag_last", lambda level: 2.0)
    assert _fails(test_coarse_operators_are_the_1d_galerkin_products, 16, 3)


def test_mutant_source_term_without_the_square(monkeypatch):
    real = P.c_term

    def c_bad(u, term):
        if term == P.HEAT_NL1:
            eu = np.exp(u)
            return u + u * eu + u * np.exp(-u)
        return real(u, term)
    monkeypatch.setattr(P, "c_term", c_bad)
    assert _fails(test_manufactured_solution_second_order, W.PDE_HEAT_NL1)


def test_mutant_post_smoothing_in_the_same_colour_order(monkeypatch):
    """Red-black after the correction as before it: the cycle is no longer
    symmetric."""
    def vbad(Rhs, h, level=0):
        N = Rhs.shape[0]
        E = np.zeros_like(Rhs)
        P.gs_colour(E, Rhs, h, P.RED, level)
        P.gs_colour(E, Rhs, h, P.BLACK, level)
        if N % 2 == 0:
            E += P.prolong(vbad(P.restrict(Rhs - P.apply_A(E, h, level)), 2 * h, level + 1))
        P.gs_colour(E, Rhs, h, P.RED, level)
        P.gs_colour(E, Rhs, h, P.BLACK, level)
        return E
    monkeypatch.setattr(P, "vcycle", vbad)
    assert _fails(test_vcycle_is_symmetric_positive_definite, 12)


def test_mutant_bratu_sign(monkeypatch):
    real = P.map_rhs
    monkeypatch.setattr(P, "map_rhs", lambda pr, u, b, lam: -real(pr, u, b, lam)
                        if pr == P.BRATU else real(pr, u, b, lam))
    assert _fails(test_fixed_point_satisfies_the_discrete_equations, lambda: W.bratu2d(16))
