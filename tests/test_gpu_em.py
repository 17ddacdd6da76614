"""GPU parity of the EM workload (Sec. 5.3): the library's EM map against the
oracle's on the same samples, and AA(3) on it against the oracle iterate by
iterate until the relative residual reaches 1e-8 (the paper's tolerance),
with the same iteration count (a loose pin against the paper's 21: the
samples and starting means are this build's)."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, rel, rel_inf, to_dev

pytestmark = pytest.mark.gpu

VARIANTS = [("mgs", 0), ("cgs2", 0), ("dcgs2", 0), ("icwy", 0), ("dcgs2_lag", 0),
            ("icwy", 1 << 2)]


def em_map(prob):
    import torch
    from paper_2110_09667_amd import aa
    xd = to_dev(prob.samples)
    work = torch.empty(aa.EM_WORK_DOUBLES, dtype=torch.float64, device="cuda")

    def G(u, out):
        aa.aa_em_apply(prob.alpha, prob.sigma, xd, u, out, work)
    return G


@pytest.mark.parametrize("nsamples,replicas", [(100_000, 1000), (777, 3), (1, 1), (300_001, 17)])
def test_em_map_matches_oracle(nsamples, replicas):
    import torch
    device()
    prob = W.em_problem(nsamples=nsamples, replicas=replicas)
    G = em_map(prob)
    for mu in ((0.1, 0.4, 1.3), (-1.0, 0.25, 2.0)):
        u = np.tile(np.array(mu), replicas)
        out = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        G(to_dev(u), out)
        ref = O.G_em(prob, u)
        got = out.cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-13, atol=0), (got[:3], ref[:3])
        assert np.array_equal(got, np.tile(got[:3], replicas))


def test_em_map_argument_errors():
    import torch
    device()
    from paper_2110_09667_amd import aa
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    u = torch.zeros(7, dtype=torch.float64, device="cuda")  # not a multiple of 3
    w = torch.empty(aa.EM_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    with pytest.raises(aa.AAError):
        aa.aa_em_apply((0.3, 0.3, 0.4), (1.0, 1.0, 1.0), x, u, u, w)
    u = torch.zeros(6, dtype=torch.float64, device="cuda")
    with pytest.raises(aa.AAError):
        aa.aa_em_apply((0.3, 0.0, 0.4), (1.0, 1.0, 1.0), x, u, u, w)


@pytest.mark.parametrize("variant,flags", VARIANTS,
                         ids=["mgs", "cgs2", "dcgs2", "icwy", "dcgs2_lag", "icwy_T_transform"])
@pytest.mark.parametrize("replicas", [500_000, 50])
def test_aa_em_matches_oracle_to_tolerance(variant, flags, replicas):
    """n = 1.5 million (the paper's vector per GPU; grid-wide passes) and
    n = 150 (one-workgroup step where the variant has one), m = 3."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    prob = W.em_problem(replicas=replicas)
    tol, cap = 1e-8, 100
    xs_ref, st, res = O.run_aa(lambda u: O.G_em(prob, u), prob.u0(), 3, variant, cap, tol=tol,
                               flags=flags)
    its_ref = len(res) - 1  # AA steps taken before the stop test held
    G = em_map(prob)
    ctx = aa.AAContext(prob.n, 3, variant, flags)
    x = to_dev(prob.u0())
    g = torch.empty_like(x)
    worst, its = 0.0, 0
    for i in range(cap + 1):
        G(x, g)
        if i >= 1:
            f = torch.linalg.norm(g - x).item()
            if f <= tol * ctx.info().res0_norm:
                break
        ctx.step(x, g, x)
        its += 1
        if i + 1 < len(xs_ref):
            xi = x.cpu().numpy()
            worst = max(worst, rel(xi, xs_ref[i + 1]), rel_inf(xi, xs_ref[i + 1]))
    assert ctx.info().status == 0
    assert worst <= 1e-10, worst
    assert its == its_ref, (its, its_ref)
    assert 12 <= its <= 30
    print(f"\nEM {variant} flags={flags} n={prob.n}: {its} iterations to 1e-8 "
          f"(oracle {its_ref}), max rel diff {worst:.1e}")
