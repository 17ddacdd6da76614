"""Seeded synthetic inputs for the Anderson-acceleration workloads.

This module is the only code shared by the FP64 CPU oracle (``oracle/``) and
the HIP library (``paper_2110_09667_amd/``).  It holds the random-number
generator and the workload recipes (grid sizes, spacing, relaxation weight,
right-hand sides); it holds none of the arithmetic of Anderson acceleration,
Gram-Schmidt or Givens rotations.

Generator
---------
Every stream is counter based.  Element ``i`` of stream ``(seed, stream)`` is

    u_i = (mix(base + i) >> 11) * 2**-53,      base = mix(mix(seed) + stream)

where ``mix(z)`` is the output function of SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
``z + 0x9E3779B97F4A7C15`` (all arithmetic modulo 2**64).  ``u_i`` lies in
[0, 1).  Normal deviates use the Box-Muller cosine branch on the pair
(u_{2i}, u_{2i+1}):  z_i = sqrt(-2 log(1 - u_{2i})) * cos(2 pi u_{2i+1}).

The HIP library carries its own implementation of the same definition for
inputs too large to generate on the host; uniforms agree bit for bit, normals
agree to a few ulps (the transcendental functions differ).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 2.0 ** -53


def mix(z):
    """SplitMix64 output function of ``z + golden`` (uint64, wraps mod 2**64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_base(seed: int, stream: int) -> int:
    """64-bit counter origin of stream ``(seed, stream)``."""
    s = int(mix(np.uint64(seed % 2**64)))
    return int(mix(np.uint64((s + stream) % 2**64)))


def uniform(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` uniforms in [0, 1) from elements ``offset .. offset+n-1``."""
    base = stream_base(seed, stream)
    ctr = np.arange(offset, offset + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = ctr + np.uint64(base)
    return (mix(ctr) >> np.uint64(11)).astype(np.float64) * _TWO_M53


def normal(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` standard normals (Box-Muller, cosine branch)."""
    u = uniform(seed, stream, 2 * n, 2 * offset)
    u1, u2 = u[0::2], u[1::2]
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------------------
# Model problems: G(u) = u - omega * (A u + c u^3 - f) on a d-dimensional
# Dirichlet grid of s points per side, A the standard (2d+1)-point Laplacian
# scaled by 1/h^2 with h = 1/(s+1).  The linear 1D case is c = 0, f = b.
# --------------------------------------------------------------------------

def laplacian_lambda_max(d: int, s: int) -> float:
    """Largest eigenvalue of the Dirichlet (2d+1)-point Laplacian, closed form.

    Each 1D factor tridiag(-1, 2, -1)/h^2 has eigenvalues
    (4/h^2) sin^2(j pi / (2(s+1))), j = 1..s; the largest is j = s, i.e.
    (4/h^2) cos^2(pi / (2(s+1))).  The d-dimensional operator is a Kronecker
    sum, so its largest eigenvalue is d times that.
    """
    h = 1.0 / (s + 1)
    return d * (4.0 / (h * h)) * math.cos(math.pi / (2.0 * (s + 1))) ** 2


def laplacian_lambda_min(d: int, s: int) -> float:
    h = 1.0 / (s + 1)
    return d * (4.0 / (h * h)) * math.sin(math.pi / (2.0 * (s + 1))) ** 2


@dataclass
class StencilProblem:
    """One instance of G(u) = u - omega (A u + c u^3 - f)."""

    d: int            # grid dimension (1, 2 or 3)
    s: int            # points per side; n = s**d
    c: float          # coefficient of the cubic term (0 for the linear case)
    f: np.ndarray     # right-hand side, length n
    omega: float = 0.0
    h: float = 0.0

    def __post_init__(self):
        self.h = 1.0 / (self.s + 1)
        if self.omega == 0.0:
            self.omega = 0.9 / laplacian_lambda_max(self.d, self.s)

    @property
    def n(self) -> int:
        return self.s ** self.d


# Seeds of the named workloads.
SEED_POISSON1D_B = 1
SEED_POISSON3D_F = 2
SEED_QR_Q = 3
SEED_QR_V = 4
SEED_EM = 5
SEED_TRAIN_BASE = 1_000_000


def poisson1d(n: int = 4096, seed: int = SEED_POISSON1D_B) -> StencilProblem:
    """Linear 1D Poisson fixed point G(x) = x - omega (A x - b), b ~ U[-1, 1]."""
    b = 2.0 * uniform(seed, 0, n) - 1.0
    return StencilProblem(d=1, s=n, c=0.0, f=b)


def nonlinear3d(s: int = 256, seed: int = SEED_POISSON3D_F) -> StencilProblem:
    """3D nonlinear fixed point G(u) = u - omega (A u + u^3 - f), f ~ U[0, 1]."""
    f = uniform(seed, 0, s ** 3)
    return StencilProblem(d=3, s=s, c=1.0, f=f)


@dataclass
class BatchInstance:
    seed: int
    s: int
    m: int
    c: float

    @property
    def n(self) -> int:
        return self.s * self.s


def batch_instance(seed: int, s_lo: int = 32, s_hi: int = 512, m_lo: int = 3,
                   m_hi: int = 20) -> BatchInstance:
    """Parameters of one 2D instance: s log-uniform on [s_lo, s_hi], m uniform
    on {m_lo..m_hi}, c ~ U[0, 1] (stream 0 of the instance seed)."""
    u = uniform(seed, 0, 3)
    s = int(round(s_lo * (s_hi / s_lo) ** u[0]))
    m = m_lo + int(math.floor((m_hi - m_lo + 1) * u[1]))
    return BatchInstance(seed=seed, s=s, m=min(m, m_hi), c=float(u[2]))


def batch_problem(inst: BatchInstance) -> StencilProblem:
    """The 2D problem of a batch instance; f ~ U[0, 1] from stream 1."""
    return StencilProblem(d=2, s=inst.s, c=inst.c, f=uniform(inst.seed, 1, inst.n))


def batch_table(count: int = 4096, first_seed: int = 0, **kw) -> list[BatchInstance]:
    return [batch_instance(first_seed + j, **kw) for j in range(count)]


# --------------------------------------------------------------------------
# Expectation-maximization of the means of a univariate normal mixture
# (the paper's Sec. 5.3): three components with known proportions alpha and
# standard deviations sigma, unknown means, unlabeled samples.  The AA vector
# holds R replicas of the three means; the map updates the means of the
# first replica and writes the result to every replica (Sec. 5.3 estimates one
# set of means redundantly in every entry).  This module only draws the
# samples and the starting point; the map itself lives in the oracle and in
# the library.
# --------------------------------------------------------------------------

@dataclass
class EMProblem:
    samples: np.ndarray          # N draws from the mixture
    alpha: tuple = (0.3, 0.3, 0.4)
    sigma: tuple = (1.0, 1.0, 1.0)
    mu_true: tuple = (0.0, 0.5, 1.0)
    replicas: int = 1

    @property
    def n(self) -> int:
        return 3 * self.replicas

    def u0(self) -> np.ndarray:
        """Starting means: the samples' 1/6, 1/2 and 5/6 quantiles (distinct,
        ordered, no constant chosen by hand), replicated."""
        q = np.quantile(self.samples, [1.0 / 6.0, 0.5, 5.0 / 6.0])
        return np.tile(q, self.replicas)


def em_problem(nsamples: int = 100_000, replicas: int = 500_000, seed: int = SEED_EM,
               alpha=(0.3, 0.3, 0.4), sigma=(1.0, 1.0, 1.0), mu=(0.0, 0.5, 1.0)) -> EMProblem:
    """Samples of the mixture sum_i alpha_i N(mu_i, sigma_i^2): component
    i of sample k from uniform k of stream 0 (the first i with u < alpha_0 +
    .. + alpha_i), the value mu_i + sigma_i z_k with z_k normal k of stream 1.
    Defaults: the paper's poorly separated mixture, 100,000 samples, 500,000
    replicas (1.5 million entries, the paper's vector per GPU)."""
    u = uniform(seed, 0, nsamples)
    cum = np.cumsum(alpha)
    comp = np.searchsorted(cum, u, side="right")
    comp = np.minimum(comp, len(alpha) - 1)
    z = normal(seed, 1, nsamples)
    x = np.asarray(mu)[comp] + np.asarray(sigma)[comp] * z
    return EMProblem(samples=x, alpha=tuple(alpha), sigma=tuple(sigma), mu_true=tuple(mu),
                     replicas=replicas)


# --------------------------------------------------------------------------
# 2D heat equation with a nonlinear term (Sec. 5.1) and the 2D Bratu problem
# (Sec. 5.2) on the unit square: N x N interior points (x fastest),
# h = 1 / (N + 1), zero Dirichlet values.  This module only tabulates the
# source term of the manufactured solution; the fixed-point maps (a linear
# Poisson solve per evaluation) live in the oracle and in the library.
# --------------------------------------------------------------------------

PDE_HEAT_NL1, PDE_HEAT_NL2, PDE_BRATU = 1, 2, 3


@dataclass
class PDE2DProblem:
    problem: int                 # PDE_HEAT_NL1, PDE_HEAT_NL2 or PDE_BRATU
    N: int                       # interior points per side; n = N * N
    m: int                       # window the paper uses for this problem
    b: np.ndarray | None = None  # heat: f at the grid points (None for Bratu)
    lam: float = 6.7             # Bratu parameter
    tol: float = 1e-10           # nonlinear and linear tolerance of the paper

    @property
    def n(self) -> int:
        return self.N * self.N

    @property
    def h(self) -> float:
        return 1.0 / (self.N + 1)

    def u0(self) -> np.ndarray:
        return np.zeros(self.n)


def grid_points(N: int):
    """Coordinates (X, Y) of the interior points, (N, N) arrays, x fastest."""
    t = np.arange(1, N + 1, dtype=np.float64) / (N + 1)
    return np.meshgrid(t, t, indexing="xy")


def heat_exact(N: int) -> np.ndarray:
    """u(x, y) = sin^2(pi x) sin^2(pi y) at the interior points (flat)."""
    X, Y = grid_points(N)
    return (np.sin(np.pi * X) ** 2 * np.sin(np.pi * Y) ** 2).reshape(-1)


def heat_source(N: int, term: int) -> np.ndarray:
    """f = u_xx + u_yy + c(u) of the manufactured solution u = sin^2(pi x)
    sin^2(pi y), evaluated at the grid points (flat): the two second
    derivatives 2 pi^2 (cos^2 - sin^2) times the other factor, and the
    reaction term of the chosen problem at u."""
    X, Y = grid_points(N)
    sx, cx = np.sin(np.pi * X), np.cos(np.pi * X)
    sy, cy = np.sin(np.pi * Y), np.cos(np.pi * Y)
    lap = 2 * np.pi ** 2 * (cx * cx - sx * sx) * sy * sy + 2 * np.pi ** 2 * (cy * cy - sy * sy) * sx * sx
    u = sx * sx * sy * sy
    if term == PDE_HEAT_NL1:
        eu = np.exp(u)
        cu = u + u * eu + u * np.exp(-u) + (u - eu) ** 2
    elif term == PDE_HEAT_NL2:
        cu = 100.0 * (u - u * u)
    else:
        raise ValueError(term)
    return (lap + cu).reshape(-1)


def heat2d(N: int = 1024, term: int = PDE_HEAT_NL1) -> PDE2DProblem:
    """Sec. 5.1 on a 1024 x 1024 grid: term 1 with m = 5, term 2 with m = 10."""
    return PDE2DProblem(problem=term, N=N, m=5 if term == PDE_HEAT_NL1 else 10,
                        b=heat_source(N, term))


def bratu2d(N: int = 1024, lam: float = 6.7) -> PDE2DProblem:
    """Sec. 5.2 on a 1024 x 1024 grid, lambda = 6.7, m = 30."""
    return PDE2DProblem(problem=PDE_BRATU, N=N, m=30, lam=lam)
