"""Pins of the oracle's learned-candidate formula (used to check the GPU
training gradient).  With delta gamma = 0 the candidate is the damped AA
step: beta = 1 gives the plain AA iterate x_{i+1}; beta = 0 gives the
undamped base point x_i - X_i gamma, X_i = [Delta x_{i-m_i} .. Delta x_{i-1}]
(since G_i - F_i = X_i and Q R = F_i)."""
import numpy as np

import aa_workloads as W
import oracle as O


def run_to(prob, m, variant, iters):
    st = O.AA(prob.n, m, variant)
    x = np.zeros(prob.n)
    xs, gs = [], []
    for _ in range(iters):
        g = O.G_stencil(prob, x)
        xs.append(x.copy())
        gs.append(g.copy())
        x = st.step(x, g)
    return st, xs, gs, x


def test_candidate_beta_one_is_plain_step():
    prob = W.batch_problem(W.BatchInstance(seed=3, s=12, m=4, c=0.5))
    for variant in ("mgs", "icwy"):
        st, xs, gs, x_next = run_to(prob, 4, variant, 9)
        xc = O.learned_candidate(st, gs[-1], np.zeros(20), 1.0)
        assert np.allclose(xc, x_next, rtol=0, atol=1e-14 * np.abs(x_next).max())


def test_candidate_beta_zero_is_undamped_base_point():
    prob = W.batch_problem(W.BatchInstance(seed=4, s=10, m=3, c=0.2))
    st, xs, gs, _ = run_to(prob, 3, "cgs2", 8)
    i = len(xs) - 1
    mi = st.m_i
    X = np.stack([xs[j + 1] - xs[j] for j in range(i - mi, i)], 1)
    ref = xs[i] - X @ st.gamma_k()
    xc = O.learned_candidate(st, gs[-1], np.zeros(20), 0.0)
    assert np.allclose(xc, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_loss_is_log_residual_ratio():
    prob = W.batch_problem(W.BatchInstance(seed=5, s=9, m=5, c=0.9))
    st, xs, gs, x_next = run_to(prob, 5, "dcgs2", 7)
    out = np.zeros(21)
    out[20] = 40.0  # beta = 1 to double precision
    L = O.learned_loss(prob, st, gs[-1], out)
    r = O.G_stencil(prob, x_next) - x_next
    assert abs(L - np.log(r @ r / (st.f @ st.f))) < 1e-12
