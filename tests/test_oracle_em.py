"""Pins of the oracle's EM map (Sec. 5.3: the means of a three-component
univariate normal mixture with known proportions and deviations).

* the update against the formula evaluated independently, sample by sample
  with math.exp and exactly rounded sums (math.fsum);
* EM never decreases the log-likelihood (Dempster, Laird and Rubin 1977);
* translation and permutation equivariance of the update;
* well separated components: the update returns each cluster's sample mean;
* the replicated vector: every triple receives the update of the first;
* AA(3) reaches 1e-8 in the same number of iterations for every variant,
  close to the 21 the paper reports (a loose pin: the samples and the
  starting means are this build's)."""
import math

import numpy as np
import pytest

import aa_workloads as W
import oracle as O

VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy", "dcgs2_lag"]


def small(nsamples=2000, replicas=2, **kw):
    return W.em_problem(nsamples=nsamples, replicas=replicas, **kw)


def formula(prob, mu):
    num, den = [[], [], []], [[], [], []]
    for x in prob.samples:
        p = [a / (math.sqrt(2 * math.pi) * s) * math.exp(-(x - m) ** 2 / (2 * s * s))
             for a, s, m in zip(prob.alpha, prob.sigma, mu)]
        t = math.fsum(p)
        for i in range(3):
            num[i].append(x * p[i] / t)
            den[i].append(p[i] / t)
    return np.array([math.fsum(num[i]) / math.fsum(den[i]) for i in range(3)])


def loglik(prob, mu):
    x = prob.samples[:, None]
    a, s = np.asarray(prob.alpha), np.asarray(prob.sigma)
    p = a / (np.sqrt(2 * np.pi) * s) * np.exp(-(x - mu) ** 2 / (2 * s * s))
    return float(np.sum(np.log(p.sum(1))))


@pytest.mark.parametrize("mu", [(0.1, 0.4, 1.3), (-1.0, 0.25, 2.0), (0.5, 0.5, 0.6)])
def test_update_matches_formula(mu):
    prob = small()
    u = np.tile(np.array(mu), prob.replicas)
    g = O.G_em(prob, u)
    ref = formula(prob, mu)
    assert np.allclose(g[:3], ref, rtol=1e-14, atol=0)


def test_replicas_receive_the_first_triples_update():
    prob = small(replicas=5)
    u = np.tile(np.array([0.1, 0.4, 1.3]), 5)
    u[3:] += np.linspace(1, 2, 12)  # other replicas do not enter
    g = O.G_em(prob, u)
    assert np.array_equal(g, np.tile(g[:3], 5))
    assert np.array_equal(g[:3], O.G_em(prob, np.tile(u[:3], 5))[:3])


def test_em_never_decreases_the_likelihood():
    prob = small(nsamples=5000)
    for mu0 in ((-1.0, 0.25, 2.0), (0.0, 1.0, 2.0), (0.9, 0.5, 0.1)):
        mu = np.array(mu0)
        ll = loglik(prob, mu)
        for _ in range(25):
            mu = O.G_em(prob, np.tile(mu, prob.replicas))[:3]
            ll2 = loglik(prob, mu)
            assert ll2 >= ll - 1e-9 * abs(ll)
            ll = ll2


def test_translation_and_permutation_equivariance():
    prob = small()
    mu = np.array([0.1, 0.4, 1.3])
    g = O.G_em(prob, np.tile(mu, 2))[:3]
    c = 3.25
    shifted = W.EMProblem(samples=prob.samples + c, alpha=prob.alpha, sigma=prob.sigma, replicas=2)
    gs = O.G_em(shifted, np.tile(mu + c, 2))[:3]
    assert np.allclose(gs, g + c, rtol=0, atol=1e-12)
    perm = [2, 0, 1]
    pp = W.EMProblem(samples=prob.samples, alpha=tuple(np.array(prob.alpha)[perm]),
                     sigma=tuple(np.array(prob.sigma)[perm]), replicas=2)
    gp = O.G_em(pp, np.tile(mu[perm], 2))[:3]
    assert np.allclose(gp, g[perm], rtol=1e-14, atol=0)


def test_separated_components_give_cluster_means():
    prob = W.em_problem(nsamples=3000, replicas=1, mu=(-60.0, 0.0, 60.0))
    x = prob.samples
    clusters = [x[x < -30], x[(x > -30) & (x < 30)], x[x > 30]]
    g = O.G_em(prob, np.array([-55.0, 2.0, 58.0]))
    for i in range(3):
        assert abs(g[i] - math.fsum(clusters[i]) / len(clusters[i])) <= 1e-12 * 60


def test_aa_converges_like_the_paper_reports():
    prob = W.em_problem(replicas=4)
    counts = []
    for v in VARIANTS:
        xs, st, res = O.run_aa(lambda u: O.G_em(prob, u), prob.u0(), 3, v, 200, tol=1e-8,
                               record=False)
        assert res[-1] <= 1e-8 * st.res0_norm
        counts.append(len(res) - 1)  # AA steps before the stop test held
    assert len(set(counts)) == 1, counts
    assert 12 <= counts[0] <= 30, counts
