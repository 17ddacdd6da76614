"""The batched path's two tilings of the persistent kernel and its split path
(large instances leave the persistent kernel for the grid-wide passes once
few instances are active), each against the CPU oracle run instance by
instance on the same seeded 2D workloads."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, rel

pytestmark = pytest.mark.gpu

VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy"]


def table(count, seed0, s_lo=5, s_hi=80):
    insts = W.batch_table(count, first_seed=seed0, s_lo=s_lo, s_hi=s_hi, m_lo=3, m_hi=12)
    return insts, [W.batch_problem(i) for i in insts]


@pytest.mark.parametrize("pairs", [2, 4])
@pytest.mark.parametrize("variant", VARIANTS)
def test_tiles_match_oracle(variant, pairs):
    """Tiles of 1024 and 2048 rows per workgroup: 15 iterations against the
    oracle (the tiling changes only the order of the partial sums)."""
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(10, 77)
    iters = 15
    b = aa.AABatch(probs, [i.m for i in insts], variant, tol=0.0, max_iter=10**9)
    b.set_tiles(pairs)
    b.run(iters + 1)
    states, _ = b.read()
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, _, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant, iters)
        assert rel(b.x[j].cpu().numpy(), xs[-1]) <= 1e-10, (j, inst)
        assert states[j].iter == iters + 1 and states[j].status == 0


def test_tiles_rejects_other_values():
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(2, 5)
    b = aa.AABatch(probs, [i.m for i in insts], "icwy", tol=0.0, max_iter=10**9)
    for bad in (0, 1, 3, 8):
        with pytest.raises(RuntimeError):
            b.set_tiles(bad)
    with pytest.raises(RuntimeError):
        b.set_split(-1, 0)


@pytest.mark.parametrize("flags", [0, "rhs+delete"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_split_matches_oracle(variant, flags):
    """Instances with n >= 1600 move to the grid-wide passes after their
    first iterations (at a run boundary, mid-window for some, with a full
    window for others); the rest stay in the persistent kernel.  Every
    instance's iterate after 15 iterations matches the oracle, and so do its
    counters."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    f = 0 if flags == 0 else aa.FUSE_RHS | aa.FUSE_DELETE
    insts, probs = table(10, 140)
    assert any(p.n >= 1600 for p in probs) and any(p.n < 1600 for p in probs)
    iters = 15
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = aa.AABatch(probs, [i.m for i in insts], variant, flags=f, tol=0.0,
                       max_iter=10**9, stream=stream)
        b.set_split(1600, 64)
        b.run(5)          # iterations 0..4 in the persistent kernel
        assert b.split_count() == 0
        b.run(3)          # split from here on (the policy runs at each run)
        assert b.split_count() == sum(1 for p in probs if p.n >= 1600)
        b.run(iters + 1 - 8)
        states, active = b.read()
    assert active == len(insts)
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, st, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant, iters)
        assert rel(b.x[j].cpu().numpy(), xs[-1]) <= 1e-10, (j, inst, p.n)
        assert states[j].iter == iters + 1 and states[j].k == min(inst.m, iters)
        assert states[j].m_i == min(inst.m, iters)
        assert states[j].status == 0
        assert abs(states[j].res_norm - st.res_norm) <= 1e-10 * st.res0_norm


@pytest.mark.parametrize("variant", ["icwy", "cgs2"])
def test_split_stops_at_tolerance_and_cap(variant):
    """The split instances stop by the batch's rule: the first i with
    ||f_i|| <= 1e-8 ||f_0|| (within one iteration of the oracle's), or at
    the iteration cap; an instance that stopped keeps its iterate while the
    others go on."""
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(8, 300, s_lo=30, s_hi=70)
    cap = 250
    b = aa.AABatch(probs, [i.m for i in insts], variant, tol=1e-8, max_iter=cap)
    b.set_split(1, 64)  # every instance splits after its first run
    b.run(2)
    b.run(1)
    assert b.split_count() == len(insts)
    for _ in range(cap // 10 + 2):
        b.run(10)
        _, active = b.read()
        if active == 0:
            break
    states, active = b.read()
    assert active == 0
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, st, res = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, variant,
                               iters=cap, tol=1e-8)
        oracle_stop = len(res) - 1
        assert 1 <= states[j].stop_iter <= cap
        if oracle_stop < cap - 1:
            assert abs(states[j].stop_iter - oracle_stop) <= 1, (j, states[j].stop_iter,
                                                                 oracle_stop)
            assert states[j].res_norm <= 1e-8 * states[j].res0_norm
            k = states[j].stop_iter
            assert rel(b.x[j].cpu().numpy(), xs[min(k, len(xs) - 1)]) <= 1e-6
        else:
            assert states[j].stop_iter >= cap - 1
        assert states[j].g_evals == states[j].stop_iter + 1


def test_split_off_returns_instances_to_the_persistent_kernel():
    """Splitting, then switching the policy off mid-run (every instance back
    in the persistent kernel, graph replay on): the iterates still match the
    oracle."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    insts, probs = table(6, 410)
    iters = 14
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = aa.AABatch(probs, [i.m for i in insts], "icwy", tol=0.0, max_iter=10**9,
                       stream=stream)
        b.set_split(1, 64)
        b.run(3)
        b.run(5)
        assert b.split_count() == len(insts)
        b.set_split(0, 0)
        assert b.split_count() == 0
        b.run(iters + 1 - 8)
        states, _ = b.read()
    for j, (inst, p) in enumerate(zip(insts, probs)):
        xs, _, _ = O.run_aa(lambda u: O.G_stencil(p, u), np.zeros(p.n), inst.m, "icwy", iters)
        assert rel(b.x[j].cpu().numpy(), xs[-1]) <= 1e-10, (j, inst)
        assert states[j].iter == iters + 1
