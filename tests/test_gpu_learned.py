"""The learned-guarded batched step (an addition on top of the paper's
method): a network that proposes no correction and beta = 1 reproduces plain
batched AA bit for bit; the guard accepts only candidates that lower the
fixed-point residual; the training gradient with respect to the network
outputs (back-propagated through G by the adjoint stencil) matches central
finite differences of the oracle's one-step loss on the oracle's own state."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, rel

pytestmark = pytest.mark.gpu

VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy"]


def table(count, seed0, s_hi=48, m_hi=12):
    insts = W.batch_table(count, first_seed=seed0, s_lo=6, s_hi=s_hi, m_lo=3, m_hi=m_hi)
    return insts, [W.batch_problem(i) for i in insts]


def const_params(P, bias_out):
    """All weights zero; the last layer's bias = bias_out (21 values): the
    network then outputs bias_out for every input."""
    p = np.zeros(P, dtype=np.float32)
    p[-64:-64 + 21] = bias_out
    return p


@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_network_reproduces_plain_bitwise(variant):
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(10, 400)
    ms = [i.m for i in insts]
    plain = aa.AABatch(probs, ms, variant, tol=0.0, max_iter=10**9)
    plain.set_schedule(use_graph=False)
    lrn = aa.AABatch(probs, ms, variant, flags=aa.BATCH_LEARNED, tol=0.0, max_iter=10**9)
    net = aa.AAMlp(len(insts))
    bias = np.zeros(21, dtype=np.float32)
    bias[20] = 40.0  # beta = 1 in double precision: no damping, no correction
    net.set_params(const_params(net.P, bias))
    iters = 14
    acc_prev = None
    for t in range(iters):
        if t == iters - 1:
            acc_prev = [s.accepted for s in lrn.read()[0]]
        plain.run(1)
        lrn.run_learned(net, 1)
    sp, _ = plain.read()
    sl, _ = lrn.read()
    for j in range(len(insts)):
        assert np.array_equal(plain.x[j].cpu().numpy(), lrn.x[j].cpu().numpy()), j
        assert sp[j].iter == sl[j].iter == iters
        assert sp[j].res_norm == sl[j].res_norm
        # one G evaluation per candidate (every call after the first), and the
        # evaluation at x_{i+1} is saved whenever the candidate was taken
        assert sp[j].g_evals == iters
        assert sl[j].g_evals == iters + (iters - 1) - acc_prev[j], (j, sl[j].g_evals)


def net_with_outputs(aa, count, o, seed=0):
    """A network whose output is the constant o (21 values)."""
    net = aa.AAMlp(count, seed=seed)
    net.set_params(const_params(net.P, np.asarray(o, dtype=np.float32)))
    return net


@pytest.mark.parametrize("variant", ["icwy", "cgs2"])
def test_guard_accepts_only_residual_decrease(variant):
    """A random network: whenever the guard takes the candidate, the residual
    formed at the next iteration, ||G(x_c) - x_c||, is below ||f_i||."""
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(12, 500)
    b = aa.AABatch(probs, [i.m for i in insts], variant, flags=aa.BATCH_LEARNED, tol=0.0,
                   max_iter=10**9)
    net = aa.AAMlp(len(insts), seed=77)
    hist = [b.read()[0]]
    for _ in range(14):
        b.run_learned(net, 1)
        hist.append(b.read()[0])
    checked = 0
    for t in range(1, len(hist) - 1):
        for j in range(len(insts)):
            if hist[t][j].accepted > hist[t - 1][j].accepted:
                assert hist[t + 1][j].res_norm < hist[t][j].res_norm * (1 + 1e-12), (t, j)
                checked += 1
    assert all(s.iter == 14 for s in hist[-1])
    assert checked > 0  # the guard accepted candidates, and each one was checked


@pytest.mark.parametrize("variant", VARIANTS)
def test_guarded_step_matches_oracle(variant):
    """Plain steps (a network with beta = 1 and no correction), then one step
    with fixed outputs: the new iterate is the oracle's candidate when its
    residual is clearly below ||f_i||, the oracle's AA iterate when clearly
    above, and the guard's decision agrees with the oracle's."""
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(8, 800, s_hi=40, m_hi=10)
    b = aa.AABatch(probs, [i.m for i in insts], variant, flags=aa.BATCH_LEARNED, tol=0.0,
                   max_iter=10**9)
    o0 = np.zeros(21)
    o0[20] = 40.0
    plain = net_with_outputs(aa, len(insts), o0)
    K = 11
    b.run_learned(plain, K - 1)
    o = np.zeros(21)
    o[:20] = 0.05 * np.cos(np.arange(20))
    o[20] = 1.5
    net = net_with_outputs(aa, len(insts), o)
    o = o.astype(np.float32).astype(np.float64)
    before, _ = b.read()
    b.run_learned(net, 1)
    after, _ = b.read()
    decided = 0
    for j, (inst, p) in enumerate(zip(insts, probs)):
        st = O.AA(p.n, inst.m, variant)
        x = np.zeros(p.n)
        for _ in range(K):
            g = O.G_stencil(p, x)
            x_next = st.step(x, g)
            if _ < K - 1:
                x = x_next
        dg = np.zeros(20)
        dg[: st.m_i] = o[: st.m_i]
        xc = O.learned_candidate(st, g, dg, 1.0 / (1.0 + np.exp(-o[20])))
        r = O.G_stencil(p, xc) - xc
        ratio = np.linalg.norm(r) / st.res_norm
        took = after[j].accepted - before[j].accepted
        got = b.x[j].cpu().numpy()
        if ratio < 1 - 1e-6:
            assert took == 1, (j, ratio)
            assert rel(got, xc) <= 1e-10, (j, rel(got, xc))
            decided += 1
        elif ratio > 1 + 1e-6:
            assert took == 0, (j, ratio)
            assert rel(got, x_next) <= 1e-10, (j, rel(got, x_next))
            decided += 1
        assert after[j].iter == K
        assert abs(after[j].res_norm - st.res_norm) <= 1e-10 * st.res0_norm
    assert decided == len(insts)


@pytest.mark.parametrize("variant", ["icwy", "mgs"])
def test_training_gradient_matches_finite_differences(variant):
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(3, 600, s_hi=24, m_hi=8)
    b = aa.AABatch(probs, [i.m for i in insts], variant, flags=aa.BATCH_LEARNED, tol=0.0,
                   max_iter=10**9)
    net = aa.AAMlp(len(insts))
    o = np.zeros(21)
    o[:20] = 0.02 * (np.arange(20) % 5 - 2)
    o[20] = 0.7
    net.set_params(const_params(net.P, o.astype(np.float32)))
    o = o.astype(np.float32).astype(np.float64)   # what the network returns
    K = 9
    b.train(net, K, lr=0.0)  # lr = 0: the network stays fixed
    states, _ = b.read()
    _, outs, douts = b.read_learning()
    scale = 1.0 / len(insts)
    for j, (inst, p) in enumerate(zip(insts, probs)):
        assert np.allclose(outs[j], o, rtol=0, atol=0)
        st = O.AA(p.n, inst.m, variant)
        x = np.zeros(p.n)
        for _ in range(K):
            g = O.G_stencil(p, x)
            x_next = st.step(x, g)
            if _ < K - 1:
                x = x_next
        mi = st.m_i
        L0 = O.learned_loss(p, st, g, o)
        assert abs(states[j].loss - L0) <= 1e-8 * max(1.0, abs(L0))
        h = 1e-6
        for k in list(range(mi)) + [20]:
            e = np.zeros(21)
            e[k] = h
            fd = (O.learned_loss(p, st, g, o + e) - O.learned_loss(p, st, g, o - e)) / (2 * h)
            got = douts[j][k] / scale
            assert abs(got - fd) <= 1e-4 * max(abs(fd), 1e-3), (j, k, got, fd)
        assert np.all(douts[j][mi:20] == 0.0)


def test_training_runs_and_changes_the_network():
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(32, 700, s_hi=40, m_hi=12)
    b = aa.AABatch(probs, [i.m for i in insts], "icwy", flags=aa.BATCH_LEARNED, tol=0.0,
                   max_iter=10**9)
    net = aa.AAMlp(len(insts), seed=3)
    p0 = net.get_params()
    b.train(net, 20, lr=1e-3)
    p1 = net.get_params()
    states, _ = b.read()
    assert np.all(np.isfinite(p1)) and not np.array_equal(p0, p1)
    assert all(np.isfinite(s.loss) for s in states)


def held_out_loss(aa, probs, ms, net, iters, variant="icwy"):
    """Mean one-step loss of the network's candidate along the plain-AA
    trajectory of the given instances (training mode with lr = 0: the network
    is not changed; every iteration takes the plain step)."""
    b = aa.AABatch(probs, ms, variant, flags=aa.BATCH_LEARNED, tol=0.0, max_iter=10**9)
    losses = []
    for t in range(iters):
        b.train(net, 1, lr=0.0)
        if t >= 1:
            losses.extend(s.loss for s in b.read()[0])
    b.close()
    return float(np.mean(losses))


def solve_counts(aa, probs, ms, net, cap, variant="icwy"):
    """Iterations and G evaluations to ||f|| <= 1e-8 ||f_0|| (plain when net is
    None, learned-guarded otherwise)."""
    flags = aa.BATCH_LEARNED if net is not None else 0
    b = aa.AABatch(probs, ms, variant, flags=flags, tol=1e-8, max_iter=cap)
    b.set_schedule(use_graph=False)
    for _ in range(cap // 25 + 2):
        if net is None:
            b.run(25)
        else:
            b.run_learned(net, 25)
        st, active = b.read()
        if active == 0:
            break
    b.close()
    return st


def test_training_generalizes_and_reports_gain(capsys):
    """Train on instances of disjoint seeds; the trained network's one-step
    loss on held-out trajectories is below the untrained network's (what the
    training optimizes), and the guarded solve with it converges every
    held-out instance.  Iterations and G evaluations to 1e-8 are printed for
    plain AA, the guard with the trained network and the guard with the
    untrained one (delta gamma = 0, beta = sigmoid(4)): the last separates
    what the damping + guard gives from what training adds."""
    device()
    from paper_2110_09667_amd import aa
    tr = W.batch_table(256, first_seed=W.SEED_TRAIN_BASE, s_lo=8, s_hi=32, m_lo=3, m_hi=10)
    te = W.batch_table(96, first_seed=7000, s_lo=8, s_hi=32, m_lo=3, m_hi=10)
    trp = [W.batch_problem(i) for i in tr]
    tep = [W.batch_problem(i) for i in te]
    trm, tem = [i.m for i in tr], [i.m for i in te]
    net0 = aa.AAMlp(256, seed=5)
    net = aa.AAMlp(256, seed=5)
    before = held_out_loss(aa, tep, tem, net0, 40)
    tb = aa.AABatch(trp, trm, "icwy", flags=aa.BATCH_LEARNED, tol=0.0, max_iter=10**9)
    for _ in range(6):           # six restarts of 60 training iterations
        tb.train(net, 60, lr=1e-3)
        tb.close()
        tb = aa.AABatch(trp, trm, "icwy", flags=aa.BATCH_LEARNED, tol=0.0, max_iter=10**9)
    after = held_out_loss(aa, tep, tem, net, 40)
    assert np.isfinite(after) and after < before, (before, after)
    cap = 3000
    sp = solve_counts(aa, tep, tem, None, cap)
    sl = solve_counts(aa, tep, tem, net, cap)
    su = solve_counts(aa, tep, tem, net0, cap)
    conv = lambda s: s.res_norm <= 1e-8 * s.res0_norm
    assert all(conv(s) for s in sp) and all(conv(s) for s in sl) and all(conv(s) for s in su)
    ip = sum(s.stop_iter for s in sp)
    il = sum(s.stop_iter for s in sl)
    gp = sum(s.g_evals for s in sp)
    gl = sum(s.g_evals for s in sl)
    acc = sum(s.accepted for s in sl)
    iu = sum(s.stop_iter for s in su)
    gu = sum(s.g_evals for s in su)
    with capsys.disabled():
        print(f"\nheld-out one-step loss {before:.3f} -> {after:.3f}; iterations plain {ip} "
              f"learned {il} ({il / ip:.3f}) untrained-guarded {iu} ({iu / ip:.3f}); "
              f"G evaluations plain {gp} learned {gl} ({gl / gp:.3f}) untrained-guarded {gu} "
              f"({gu / gp:.3f}); accepted {acc}")
