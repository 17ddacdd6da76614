"""Batched AA (many independent instances, one persistent launch per
iteration) against the CPU oracle run instance by instance on the same
seeded 2D workloads; graph replay against direct launches; stopping rule."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, rel

pytestmark = pytest.mark.gpu

VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy"]


def small_table(count=10, seed0=50):
    """2D instances with the batched workload's recipe, s scaled down so the
    oracle finishes in seconds (several tiles per instance, ragged)."""
    insts = W.batch_table(count, first_seed=seed0, s_lo=5, s_hi=80, m_lo=3, m_hi=12)
    return insts, [W.batch_problem(i) for i in insts]


@pytest.mark.parametrize("variant", VARIANTS)
def test_batch_matches_oracle(variant):
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = small_table()
    iters = 15
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = aa.AABatch(probs, [i.m for i in insts], variant, tol=0.0, max_iter=10**9,
                       stream=stream)
        for _ in range(iters + 1):
            b.run(1)
        states, active = b.read()
    assert active == len(insts)
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, st, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant, iters)
        got = b.x[j].cpu().numpy()
        assert rel(got, xs[-1]) <= 1e-10, (j, inst, rel(got, xs[-1]))
        assert states[j].iter == iters + 1 and states[j].k == min(inst.m, iters)
        assert states[j].status == 0
        # ||f_i|| is a difference of nearly equal vectors once converged: its
        # rounding is relative to ||f_0||, not to itself
        assert abs(states[j].res_norm - st.res_norm) <= 1e-10 * st.res0_norm


@pytest.mark.parametrize("variant", ["icwy", "mgs"])
def test_batch_graph_replay_equals_direct(variant):
    """The captured graph replayed several times (with eager reads between
    replays) gives bit-identical iterates to direct launches."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = small_table(count=24, seed0=90)
    ms = [i.m for i in insts]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bg = aa.AABatch(probs, ms, variant, tol=0.0, max_iter=10**9, stream=stream)
        bd = aa.AABatch(probs, ms, variant, tol=0.0, max_iter=10**9, stream=stream)
        bd.set_schedule(use_graph=False)
        for _ in range(4):
            bg.run(3)
            bd.run(3)
            sg, _ = bg.read()
            sd, _ = bd.read()
            for j in range(len(insts)):
                assert np.array_equal(bg.x[j].cpu().numpy(), bd.x[j].cpu().numpy())
                assert sg[j].iter == sd[j].iter


def test_batch_schedule_does_not_change_results():
    """Natural order and a different number of persistent workgroups give the
    same iterates (each instance is owned by one workgroup; its arithmetic
    does not depend on the schedule)."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = small_table(count=16, seed0=7)
    ms = [i.m for i in insts]
    runs = []
    for grid, order in ((0, 0), (3, 1), (64, 0)):
        b = aa.AABatch(probs, ms, "cgs2", tol=0.0, max_iter=10**9)
        b.set_schedule(grid=grid, order=order, use_graph=False)
        b.run(9)
        b.read()
        runs.append([x.cpu().numpy() for x in b.x])
    for r in runs[1:]:
        for a, c in zip(runs[0], r):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("variant", VARIANTS)
def test_batch_stops_at_tolerance(variant):
    """Each instance stops at the first i with ||f_i|| <= 1e-8 ||f_0||; the
    oracle with the same rule stops within one iteration of it (rounding can
    move a borderline residual across the threshold).  An instance that has
    not converged by max_iter stops there."""
    device()
    from paper_2110_09667_amd import aa
    insts = W.batch_table(8, first_seed=300, s_lo=5, s_hi=40, m_lo=3, m_hi=12)
    probs = [W.batch_problem(i) for i in insts]
    cap = 600
    b = aa.AABatch(probs, [i.m for i in insts], variant, tol=1e-8, max_iter=cap)
    b.set_schedule(use_graph=False)
    for _ in range(cap // 20 + 2):
        b.run(20)
        _, active = b.read()
        if active == 0:
            break
    states, active = b.read()
    assert active == 0
    for j, (inst, p) in enumerate(zip(insts, probs)):
        _, st, res = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant,
                              iters=cap, tol=1e-8)
        oracle_stop = len(res) - 1
        assert 1 <= states[j].stop_iter <= cap
        if oracle_stop < cap - 1:
            assert abs(states[j].stop_iter - oracle_stop) <= 1, (j, states[j].stop_iter, oracle_stop)
            assert states[j].res_norm <= 1e-8 * states[j].res0_norm
        else:
            assert states[j].stop_iter >= cap - 1


def test_batch_mixed_sizes_with_a_large_instance():
    """A 512^2 instance (many tiles per workgroup) among small ones."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    big = W.BatchInstance(seed=5, s=512, m=6, c=0.4)
    insts = [big] + small_table(count=5, seed0=11)[0]
    probs = [W.batch_problem(i) for i in insts]
    b = aa.AABatch(probs, [i.m for i in insts], "icwy", tol=0.0, max_iter=10**9)
    iters = 8
    b.run(iters + 1)
    b.read()
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, _, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, "icwy", iters)
        assert rel(b.x[j].cpu().numpy(), xs[-1]) <= 1e-10, j


def test_autotune_keeps_results_and_caches(tmp_path):
    """The autotuner runs real iterations under each candidate schedule: the
    iterates match those of an untuned batch after the same number of
    iterations (to rounding: the tiling sets the order of the partial sums);
    a second tuning with the same cache file runs no trial and applies the
    stored schedule."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = small_table(count=12, seed0=300)
    ms = [i.m for i in insts]
    stream = torch.cuda.Stream()
    cache = str(tmp_path / "tune.txt")
    with torch.cuda.stream(stream):
        bt = aa.AABatch(probs, ms, "icwy", tol=0.0, max_iter=10**9, stream=stream)
        bp = aa.AABatch(probs, ms, "icwy", tol=0.0, max_iter=10**9, stream=stream)
        bt.run(13)
        bp.run(13)
        best = bt.autotune(2, cache)
        assert best.trials >= 2 and best.grid >= 1 and best.ms_per_iter > 0
        done = 13 + 2 * best.trials
        bp.run(done - 13)
        st, _ = bt.read()
        sp, _ = bp.read()
        for j in range(len(insts)):
            assert st[j].iter == sp[j].iter == done
            assert rel(bt.x[j].cpu().numpy(), bp.x[j].cpu().numpy()) <= 1e-10
        again = bp.autotune(2, cache)
        assert again.trials == 0 and again.grid == best.grid and again.order == best.order
        assert again.pairs == best.pairs in (2, 4)
        assert bp.read()[0][0].iter == done
    with open(cache) as fh:
        lines = fh.read().split()
    assert len(lines) == 6 and lines[0].startswith("gfx")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("flags", ["rhs", "rhs+delete", "delete"])
def test_batch_fusion_options_match_oracle(variant, flags):
    """The batched kernel with the right-hand side folded into QRAdd and/or
    QRDelete sharing its pass with the QRAdd's first (ignored for MGS), 15
    iterations against the oracle's separate steps."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    f = {"rhs": aa.FUSE_RHS, "rhs+delete": aa.FUSE_RHS | aa.FUSE_DELETE,
         "delete": aa.FUSE_DELETE}[flags]
    insts, probs = small_table(count=8, seed0=123)
    iters = 15
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = aa.AABatch(probs, [i.m for i in insts], variant, flags=f, tol=0.0, max_iter=10**9,
                       stream=stream)
        b.run(iters + 1)
        states, _ = b.read()
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, st, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant, iters)
        assert rel(b.x[j].cpu().numpy(), xs[-1]) <= 1e-10, (j, inst)
        assert states[j].status == 0 and states[j].k == min(inst.m, iters)
