"""Pins of the model problems and of the seeded input generator.

* the oracle's stencil maps against a dense Kronecker-sum Laplacian built in
  numpy (d = 1, 2, 3) with the cubic term;
* the closed-form largest/smallest Laplacian eigenvalues against numpy's
  symmetric eigensolver;
* SplitMix64 against its published outputs for state 0 (golden file);
* the uniform and normal streams against their first moments.
"""
import os

import numpy as np
import pytest

import aa_workloads as W
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_laplacian(d, s, h):
    T = (np.diag(2.0 * np.ones(s)) - np.diag(np.ones(s - 1), 1)
         - np.diag(np.ones(s - 1), -1)) / h ** 2
    I = np.eye(s)
    if d == 1:
        return T
    if d == 2:
        return np.kron(I, T) + np.kron(T, I)
    return (np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I)
            + np.kron(np.kron(T, I), I))


@pytest.mark.parametrize("d,s", [(1, 9), (2, 5), (3, 4)])
def test_stencil_map_matches_dense(d, s):
    rng = np.random.default_rng(d)
    f = rng.uniform(size=s ** d)
    prob = W.StencilProblem(d=d, s=s, c=0.7, f=f)
    u = rng.standard_normal(s ** d)
    A = dense_laplacian(d, s, prob.h)
    ref = u - prob.omega * (A @ u + 0.7 * u ** 3 - f)
    got = O.G_stencil(prob, u)
    assert np.allclose(got, ref, rtol=0, atol=1e-14 * np.abs(A @ u).max() * prob.omega + 1e-15)
    assert np.allclose(O.laplacian(d, s, prob.h, u), A @ u, rtol=1e-13, atol=1e-9)


@pytest.mark.parametrize("d,s", [(1, 20), (2, 6), (3, 4)])
def test_lambda_closed_forms(d, s):
    ev = np.linalg.eigvalsh(dense_laplacian(d, s, 1.0 / (s + 1)))
    assert np.isclose(W.laplacian_lambda_max(d, s), ev.max(), rtol=1e-12)
    assert np.isclose(W.laplacian_lambda_min(d, s), ev.min(), rtol=1e-9)


def test_workload_constants():
    p1 = W.poisson1d()
    assert p1.n == 4096 and np.isclose(p1.omega, 1.34045e-8, rtol=1e-5)
    assert p1.f.min() >= -1.0 and p1.f.max() < 1.0
    assert np.isclose(W.laplacian_lambda_max(3, 256), 792558.39, rtol=1e-8)


def test_splitmix64_published_outputs():
    vals = [int(line, 16) for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if line.strip() and not line.startswith("#")]
    with np.errstate(over="ignore"):
        got = [int(W.mix(np.uint64(k) * W.GOLDEN)) for k in range(len(vals))]
    assert got == vals


def test_uniform_and_normal_moments():
    u = W.uniform(7, 3, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3 and abs(u.var() - 1 / 12) < 2e-3
    z = W.normal(7, 4, 200_000)
    assert abs(z.mean()) < 1e-2 and abs(z.var() - 1.0) < 1e-2
    assert abs((z ** 4).mean() - 3.0) < 0.1
    # offsets address the same counter stream
    assert np.array_equal(W.uniform(7, 3, 10, offset=5), u[5:15])
    assert np.array_equal(W.normal(7, 4, 10, offset=5), z[5:15])


def test_batch_table_ranges():
    t = W.batch_table(512)
    s = np.array([x.s for x in t])
    m = np.array([x.m for x in t])
    assert s.min() >= 32 and s.max() <= 512
    assert m.min() >= 3 and m.max() <= 20
    assert len(set(m.tolist())) == 18
