"""The stopping rule of aa_step evaluated on the device (Alg. 1's tol and
maxIters, reading A2) and the defined end of an iteration that breaks down
(reading A10), through the C ABI, on the grid-wide passes and the
one-workgroup step.

* AA_STOP_RESIDUAL: the iteration ends at the start of the first i with
  ||f_i|| <= tol ||f_0||, the same i as the oracle's driver; later calls
  leave x bitwise unchanged, also under graph replay;
* AA_STOP_STEP: ends at the first i with ||x_i - x_{i-1}|| < tol (the
  paper's test), checked against the step lengths of the oracle's run;
* the cap: iterations 1..max_iter run, then x stays;
* a repeated Delta f (the new column exactly in the span): status
  AA_EBREAKDOWN, that step returns G(x_i), later steps change nothing, and
  aa_reset restarts."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu

VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy", "dcgs2_lag"]


def drive(ctx, G, x0, calls):
    import torch
    x = to_dev(x0)
    g = torch.empty_like(x)
    xs = []
    for _ in range(calls):
        G(x, g)
        ctx.step(x, g, x)
        xs.append(x.clone())
    return xs


def em_setup():
    import torch
    from paper_2110_09667_amd import aa
    prob = W.em_problem(replicas=5000)
    xd = to_dev(prob.samples)
    work = torch.empty(aa.EM_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    return prob, (lambda u, out: aa.aa_em_apply(prob.alpha, prob.sigma, xd, u, out, work))


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("one_wg", [False, True])
def test_residual_stop_matches_oracle(variant, one_wg):
    device()
    from paper_2110_09667_amd import aa
    prob, G = em_setup()
    tol = 1e-8
    _, st, res = O.run_aa(lambda u: O.G_em(prob, u), prob.u0(), 3, variant, 100, tol=tol)
    stop_i = len(res) - 1  # the oracle's driver tests at the start of iteration i
    ctx = aa.AAContext(prob.n, 3, variant)
    ctx.set_fused_threshold((1 << 40) if one_wg else 0)
    ctx.set_stop(tol, 0, aa.STOP_RESIDUAL)
    xs = drive(ctx, G, prob.u0(), stop_i + 6)
    info = ctx.info()
    if one_wg and variant == "dcgs2_lag":
        pass  # the lagged form has no one-workgroup step: grid passes anyway
    assert info.status == 0
    assert info.stopped == aa.STOPPED_TEST, info.stopped
    assert info.stop_iter == stop_i, (info.stop_iter, stop_i)
    assert info.iter == stop_i
    # every call from iteration stop_i on returned x_stop unchanged
    final = xs[stop_i - 1].cpu().numpy()
    for x in xs[stop_i:]:
        assert np.array_equal(x.cpu().numpy(), final)
    assert rel(final, O.run_aa(lambda u: O.G_em(prob, u), prob.u0(), 3, variant,
                               stop_i - 1)[0][-1]) <= 1e-10


def test_residual_stop_under_graph_replay():
    """Steady-state iterations replayed from captured graphs keep the test:
    the replayed run ends at the same iteration, with the same iterate bit for
    bit, as the run that enqueues every pass (190 iterations here, within one
    of the oracle's count: the two trajectories part by rounding over so many
    ill-conditioned steps)."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    prob = W.nonlinear3d(s=40, seed=3)
    m, tol = 10, 1e-3
    _, _, res = O.run_aa(lambda u: O.G_stencil(prob, u), np.zeros(prob.n), m, "icwy", 400,
                         tol=tol)
    stop_ref = len(res) - 1
    assert 2 * m + 2 < stop_ref < 400  # the replayed phase is reached before the end
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        f_d = to_dev(prob.f)
        for graph in (False, True):
            ctx = aa.AAContext(prob.n, m, "icwy", stream=stream)
            ctx.set_fused_threshold(0)
            ctx.set_graph(graph)
            ctx.set_stop(tol)
            x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
            g = torch.empty_like(x)
            for _ in range(stop_ref + 6):
                aa.aa_problem_apply(3, prob.s, prob.h, prob.omega, prob.c, f_d, x, g,
                                    stream=stream)
                ctx.step(x, g, x)
            out[graph] = (ctx.info(), x.cpu().numpy())
    (i0, x0), (i1, x1) = out[False], out[True]
    assert i0.stopped == aa.STOPPED_TEST and i1.stopped == aa.STOPPED_TEST
    assert i0.stop_iter == i1.stop_iter and np.array_equal(x0, x1)
    assert abs(i0.stop_iter - stop_ref) <= 1, (i0.stop_iter, stop_ref)


@pytest.mark.parametrize("one_wg", [False, True])
def test_step_length_stop(one_wg):
    device()
    from paper_2110_09667_amd import aa
    prob = W.nonlinear3d(s=12, seed=4)
    m, iters = 5, 40
    st = O.AA(prob.n, m, "icwy")
    x = np.zeros(prob.n)
    steps = []
    for _ in range(iters + 1):
        x = st.step(x, O.G_stencil(prob, x))
        steps.append(st.step_norm)  # ||x_{i+1} - x_i|| after call i
    tol = float(np.sqrt(steps[12] * steps[13]))  # between two consecutive lengths
    # the test at the start of iteration i reads ||x_i - x_{i-1}|| = steps[i - 1]
    stop_i = next(i for i in range(1, iters) if steps[i - 1] < tol)
    ctx = aa.AAContext(prob.n, m, "icwy")
    ctx.set_fused_threshold((1 << 40) if one_wg else 0)
    ctx.set_stop(tol, 0, aa.STOP_STEP)
    f_d = to_dev(prob.f)
    G = lambda u, out: aa.aa_problem_apply(3, prob.s, prob.h, prob.omega, prob.c, f_d, u, out)
    drive(ctx, G, np.zeros(prob.n), stop_i + 4)
    info = ctx.info()
    assert info.stopped == aa.STOPPED_TEST and info.stop_iter == stop_i, (info.stop_iter, stop_i)


@pytest.mark.parametrize("one_wg", [False, True])
def test_iteration_cap(one_wg):
    device()
    from paper_2110_09667_amd import aa
    prob = W.nonlinear3d(s=12, seed=4)
    m, cap = 4, 7
    xs_ref, _, _ = O.run_aa(lambda u: O.G_stencil(prob, u), np.zeros(prob.n), m, "cgs2", cap)
    ctx = aa.AAContext(prob.n, m, "cgs2")
    ctx.set_fused_threshold((1 << 40) if one_wg else 0)
    ctx.set_stop(0.0, cap)
    f_d = to_dev(prob.f)
    G = lambda u, out: aa.aa_problem_apply(3, prob.s, prob.h, prob.omega, prob.c, f_d, u, out)
    xs = drive(ctx, G, np.zeros(prob.n), cap + 5)
    info = ctx.info()
    assert info.stopped == aa.STOPPED_CAP and info.stop_iter == cap + 1
    # calls 0..cap produce x_1..x_{cap+1}; later calls leave it
    assert rel(xs[cap].cpu().numpy(), xs_ref[cap + 1]) <= 1e-10
    for x in xs[cap + 1:]:
        assert np.array_equal(x.cpu().numpy(), xs[cap].cpu().numpy())


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("one_wg", [False, True])
def test_repeated_delta_f_ends_the_iteration(variant, one_wg):
    """The caller's G makes Delta f_1 = Delta f_0 exactly: the second QRAdd
    adds a column already in the window.  The oracle's QRAdd reports the
    breakdown on the same columns; the library latches AA_EBREAKDOWN, returns
    x_3 = G(x_2) from that step, changes nothing afterwards, and runs again
    after aa_reset."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    n, m = 3000, 4
    rng = np.random.default_rng(17)
    f0, d = rng.standard_normal(n), rng.standard_normal(n)
    ref = O.QR(n, m, variant)
    assert ref.add(d) == O.OK and ref.add(d.copy()) == O.EBREAKDOWN
    ctx = aa.AAContext(n, m, variant)
    ctx.set_fused_threshold((1 << 40) if one_wg else 0)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    xs, gs = [], []
    for i in range(5):
        f = f0 + min(i, 2) * d if i < 3 else f0 + 2 * d + rng.standard_normal(n)
        g = x + to_dev(f)  # G(x_i) = x_i + f_i, so f_i = f_0 + i d for i <= 2
        gs.append(g.clone())
        ctx.step(x, g, x)
        xs.append(x.clone())
    info = ctx.info()
    assert info.status == -3
    assert info.stopped == aa.STOPPED_BREAKDOWN and info.stop_iter == 2, (info.stopped,
                                                                         info.stop_iter)
    assert torch.equal(xs[2], gs[2])  # the breaking step returned G(x_2)
    assert torch.equal(xs[3], xs[2]) and torch.equal(xs[4], xs[2])
    ctx.reset()
    ctx.step(x, gs[0], x)  # a fresh start: x_1 = G(x_0)
    info = ctx.info()
    assert info.status == 0 and info.stopped == aa.RUNNING
    assert torch.equal(x, gs[0])
