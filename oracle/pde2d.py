"""FP64 CPU oracle of the 2D test problems of Sec. 5.1 and 5.2: the heat
equation with a nonlinear term and the Bratu problem, whose fixed-point maps
G(u) = A^{-1}(...) solve a linear Poisson system at every evaluation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing here is imported by the
HIP library or its binding, and nothing here imports them.

The paper solves the linear systems with a preconditioned conjugate gradient
whose preconditioner is a structured multigrid cycle from an external library;
that library is not available here, so the preconditioner is a geometric
multigrid V-cycle written out below (the reading is stated in each function).
Everything is plain numpy in float64, on (N, N) arrays ``U[j, i]`` with x
(index i) fastest, interior points only, h = 1 / (N + 1) and zero Dirichlet
values on the boundary.

Pins: ``tests/test_oracle_pde2d.py`` (exact solves by the discrete sine
transform and dense factorization, brute-force transfer stencils, symmetry of
the cycle, the manufactured solution's second-order convergence, the discrete
equations at the fixed point, and the iteration counts the paper reports as
loose checks).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

RED, BLACK = 0, 1
HEAT_NL1, HEAT_NL2, BRATU = 1, 2, 3


# --------------------------------------------------------------------------
# operator and multigrid pieces
# --------------------------------------------------------------------------

def diag_last(level: int) -> float:
    """h^2 times the 1D operator's last diagonal entry on multigrid level
    ``level`` (spacing 2^level h): 2 on the fine grid, 1 + 2^level below it.

    Coarse point I of a level sits at fine point 2 I + 1 of the level above,
    so the last coarse point keeps the fine grid's distance h to the right
    (top) boundary while the spacing doubles.  The 1D Galerkin operator
    R A P of the level above (R = P^T / 2 in 1D) is then the 3-point
    operator at spacing H with the last diagonal entry 1 + H / h instead of
    2: the boundary at its true distance.  The coarse 2D operator is the
    Kronecker sum of these 1D operators (5 points, symmetric)."""
    return 2.0 if level == 0 else 1.0 + 2.0 ** level


def diagonal(N: int, level: int) -> np.ndarray:
    """Diagonal of the level's 2D operator times H^2: d_x(i) + d_y(j) with
    d(i) = 2, except d(N - 1) = ``diag_last(level)``."""
    d = np.full(N, 2.0)
    d[-1] = diag_last(level)
    return d[:, None] + d[None, :]


def apply_A(U: np.ndarray, h: float, level: int = 0) -> np.ndarray:
    """A U with A = -L_h, L_h the 5-point Laplacian of Sec. 5.1 (second-order
    centred differences) with zero Dirichlet values: A is symmetric positive
    definite, so the conjugate gradient applies to it.  On a coarse level
    (spacing h = 2^level times the fine one) the diagonal of the last row
    and column follows ``diag_last``."""
    P = np.pad(U, 1)
    nb = P[1:-1, :-2] + P[1:-1, 2:] + P[:-2, 1:-1] + P[2:, 1:-1]
    return (diagonal(U.shape[0], level) * U - nb) / (h * h)


def colour_mask(N: int, colour: int) -> np.ndarray:
    """Points (i, j) with (i + j) % 2 == colour (red 0, black 1)."""
    ij = np.add.outer(np.arange(N), np.arange(N))
    return (ij % 2) == colour


def gs_colour(E: np.ndarray, Rhs: np.ndarray, h: float, colour: int, level: int = 0) -> None:
    """One Gauss-Seidel half-sweep of A E = Rhs over the points of one colour,
    in place: E_p = (h^2 Rhs_p + sum of the 4 neighbours) / diag_p (diag_p =
    4 except at the last row and column of a coarse level).  Points of one
    colour have no neighbours of that colour, so the update of all of them at
    once is the Gauss-Seidel update in any order."""
    P = np.pad(E, 1)
    nb = P[1:-1, :-2] + P[1:-1, 2:] + P[:-2, 1:-1] + P[2:, 1:-1]
    new = (h * h * Rhs + nb) / diagonal(E.shape[0], level)
    m = colour_mask(E.shape[0], colour)
    E[m] = new[m]


def prolong_1d(N: int) -> sp.csr_matrix:
    """Linear interpolation from the coarse grid to the fine grid in one
    direction, fine size N (even), coarse size N / 2.  Coarse point I sits at
    fine point 2 I + 1 (both at x = (2 I + 2) h); fine point 2 I lies between
    coarse points I - 1 and I and takes half of each, coarse point -1 being
    the boundary (zero)."""
    assert N % 2 == 0
    Nc = N // 2
    rows, cols, vals = [], [], []
    for I in range(Nc):
        rows.append(2 * I + 1); cols.append(I); vals.append(1.0)
        rows.append(2 * I); cols.append(I); vals.append(0.5)
        if 2 * I + 2 < N:
            rows.append(2 * I + 2); cols.append(I); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, Nc))


def prolong(Ec: np.ndarray) -> np.ndarray:
    """Bilinear interpolation (tensor product of ``prolong_1d``)."""
    P1 = prolong_1d(2 * Ec.shape[0])
    return P1 @ (P1 @ Ec.T).T


def restrict(Rf: np.ndarray) -> np.ndarray:
    """Full weighting, the transpose of the bilinear interpolation divided by
    4 (weights 1/4, 1/8, 1/16 at the centre, edge and corner neighbours of
    fine point (2 J + 1, 2 I + 1))."""
    P1 = prolong_1d(Rf.shape[0])
    return (P1.T @ (P1.T @ Rf.T).T) / 4.0


def levels(N: int) -> list[int]:
    """Grid sizes of the hierarchy: halve while the size is even."""
    out = [N]
    while out[-1] % 2 == 0:
        out.append(out[-1] // 2)
    return out


def vcycle(Rhs: np.ndarray, h: float, level: int = 0) -> np.ndarray:
    """One V(1,1) cycle for A E = Rhs from E = 0: red then black Gauss-Seidel
    before the coarse-grid correction, black then red after it (the reverse
    order makes the cycle a symmetric operator, as the conjugate gradient
    needs of its preconditioner).  The coarse problem is the level's
    operator at spacing 2 h (``apply_A`` with level + 1) with the restricted
    residual, solved by the same cycle recursively; on the coarsest grid
    (odd size) the cycle only smooths."""
    N = Rhs.shape[0]
    E = np.zeros_like(Rhs)
    gs_colour(E, Rhs, h, RED, level)
    gs_colour(E, Rhs, h, BLACK, level)
    if N % 2 == 0:
        res = Rhs - apply_A(E, h, level)
        Ec = vcycle(restrict(res), 2.0 * h, level + 1)
        E += prolong(Ec)
    gs_colour(E, Rhs, h, BLACK, level)
    gs_colour(E, Rhs, h, RED, level)
    return E


def pcg(rhs: np.ndarray, h: float, tol: float, max_iter: int, fixed_iters: int = -1):
    """Preconditioned conjugate gradient (Hestenes and Stiefel) for A x = rhs
    from x = 0, the preconditioner one ``vcycle``.  Stops before iteration k
    when ||r_k||_2 <= tol ||rhs||_2 (or after ``fixed_iters`` iterations when
    that is >= 0).  Returns (x, iterations, converged)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    rr0 = float(np.vdot(r, r))
    p = None
    rho_prev = 0.0
    k = 0
    while True:
        rr = float(np.vdot(r, r))
        if fixed_iters >= 0:
            if k == fixed_iters:
                return x, k, True
        elif rr <= tol * tol * rr0:
            return x, k, True
        if k == max_iter:
            return x, k, False
        z = vcycle(r, h)
        rho = float(np.vdot(r, z))
        p = z.copy() if k == 0 else z + (rho / rho_prev) * p
        q = apply_A(p, h)
        alpha = rho / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rho_prev = rho
        k += 1


# --------------------------------------------------------------------------
# the maps
# --------------------------------------------------------------------------

def c_term(u: np.ndarray, term: int) -> np.ndarray:
    """Nonlinear reaction terms of Sec. 5.1: term 1 is
    u + u e^u + u e^-u + (u - e^u)^2, term 2 is 100 (u - u^2)."""
    if term == HEAT_NL1:
        eu = np.exp(u)
        return u + u * eu + u * np.exp(-u) + (u - eu) ** 2
    if term == HEAT_NL2:
        return 100.0 * (u - u * u)
    raise ValueError(term)


def map_rhs(problem: int, u: np.ndarray, b, lam: float) -> np.ndarray:
    """Right-hand side of the linear solve inside G.  Heat (Sec. 5.1):
    L_h u + c(u) = b, so A u = c(u) - b with A = -L_h.  Bratu (Sec. 5.2):
    L_h u + lam e^u = 0, so A u = lam e^u."""
    if problem in (HEAT_NL1, HEAT_NL2):
        return c_term(u, problem) - b
    if problem == BRATU:
        return lam * np.exp(u)
    raise ValueError(problem)


def G(problem: int, u_flat: np.ndarray, N: int, b=None, lam: float = 6.7,
      tol: float = 1e-10, max_iter: int = 200, stats: dict | None = None) -> np.ndarray:
    """G(u) = A^{-1}(rhs(u)) with the linear solve by ``pcg`` to ``tol``
    (Sec. 5.1 and 5.2 use 1e-10 for the linear solver too); u and the
    result are flat vectors of N * N entries, x fastest."""
    h = 1.0 / (N + 1)
    U = np.asarray(u_flat, dtype=np.float64).reshape(N, N)
    B = None if b is None else np.asarray(b, dtype=np.float64).reshape(N, N)
    x, its, ok = pcg(map_rhs(problem, U, B, lam), h, tol, max_iter)
    if stats is not None:
        stats.setdefault("pcg_iters", []).append(its)
        stats.setdefault("pcg_converged", []).append(ok)
    return x.reshape(-1)


def residual(problem: int, u_flat: np.ndarray, N: int, b=None, lam: float = 6.7) -> np.ndarray:
    """The discrete equation's residual L_h u + c(u) - b (heat) or
    L_h u + lam e^u (Bratu), flat."""
    h = 1.0 / (N + 1)
    U = np.asarray(u_flat, dtype=np.float64).reshape(N, N)
    Lu = -apply_A(U, h)
    if problem in (HEAT_NL1, HEAT_NL2):
        return (Lu + c_term(U, problem) - np.asarray(b).reshape(N, N)).reshape(-1)
    return (Lu + lam * np.exp(U)).reshape(-1)
