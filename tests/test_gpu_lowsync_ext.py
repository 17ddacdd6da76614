"""GPU parity of the two QR-update forms Sec. 3 names besides Algs. 3-6,
against the oracle on the same inputs:

* ICWY with T updated after QRDelete by rotating the old Gram matrix, no
  reduction (AA_ICWY_T_TRANSFORM): the rotation runs without its Gram, the
  Givens kernel carries T along;
* DCGS-2 with the normalization lagged (AA_DCGS2_LAG): one reduction per
  added column, the new column normalized by Pythagoras.

Tolerances as for Algs. 3-6: single updates on well-conditioned data 1e-12,
iterates 1e-10 over 20 iterations (and the same kappa-derived bound after
them as the recycling tests)."""
import numpy as np
import pytest

import aa_workloads as W
import oracle as O
from gpu_util import device, gpu_aa_run, oracle_trajectory, rel, rel_inf, to_dev

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
# (variant, library flags, oracle flags)
FORMS = [("icwy", 1 << 2, 1 << 2), ("dcgs2_lag", 0, 0)]
IDS = ["icwy_T_transform", "dcgs2_lag"]


def graded(n, m, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (U * np.logspace(0, -np.log10(kappa), m)) @ V.T


def compare(ctx, ref, tol, t_rows):
    R, T, k = ctx.get_qr()
    assert k == ref.k
    if k == 0:
        return
    Q = ctx.basis(k).cpu().numpy()
    assert np.abs(Q - ref.Qk()).max() <= tol
    assert np.abs(R - ref.Rk()).max() <= tol * max(1.0, np.abs(ref.Rk()).max())
    if t_rows:
        Tr = ref.Tk()
        for a in range(1, k - 1):  # rows 0..k-2: the last waits for the next add
            assert np.abs(T[a, :a] - Tr[a, :a]).max() <= tol, a


@pytest.mark.parametrize("form", FORMS, ids=IDS)
@pytest.mark.parametrize("n", [6221, 257, 3])
def test_qr_add_delete_matches_oracle(form, n):
    device()
    from paper_2110_09667_amd import aa
    variant, lf, of = form
    m = 6 if n > 6 else 2
    ctx = aa.AAContext(n, m, variant, lf | aa.QR_ONLY)
    ref = O.QR(n, m, variant, of)
    cols = graded(n, 3 * m, 1e3, seed=n) if n > 3 * m else W.normal(5, 0, n * 3 * m).reshape(n, 3 * m)
    for t in range(3 * m):
        if ref.k == m:
            assert ref.delete() == 0
            ctx.qr_delete()
            compare(ctx, ref, 1e-12, variant == "icwy")
        assert ref.add(cols[:, t]) == 0
        ctx.qr_add(to_dev(cols[:, t]))
        compare(ctx, ref, 1e-12, variant == "icwy")
    assert ctx.info().status == 0
    add, dele, _ = ctx.sync_counts()
    assert (add, dele) == ref.syncs[:2], ((add, dele), ref.syncs)


@pytest.mark.parametrize("k", [4, 9, 12, 20, 33, 50, 64])
def test_T_transform_on_nonorthonormal_basis(k):
    """The rotated Gram matrix against the oracle's, on an MGS basis of a
    kappa = 1e12 matrix (orthogonality lost to ~1e-4, so every entry of T
    counts): rows 0..k-3 of the new T, R, and the next add."""
    import torch
    device()
    from paper_2110_09667_amd import aa
    n = 2 * 2048 + 77
    F = graded(n, k, 1e12, seed=300 + k)
    base = O.QR(n, k, "mgs")
    for j in range(k):
        base.add(F[:, j])
    Q0, R0 = base.Qk(), base.Rk()
    T0 = np.eye(k) + np.tril(Q0.T @ Q0, -1)
    ref = O.QR(n, k, "icwy", O.ICWY_T_TRANSFORM)
    ref.Q[:, :k], ref.R[:k, :k], ref.T[:k, :k] = Q0, R0, T0
    ref.s.k = k
    ctx = aa.AAContext(n, k, "icwy", aa.QR_ONLY | aa.ICWY_T_TRANSFORM)
    Qd = torch.from_numpy(np.ascontiguousarray(Q0.T)).cuda()
    aa.aa_qr_load(ctx.ctx, k, Qd.data_ptr(), n, R0, T0)
    assert ref.delete() == 0
    ctx.qr_delete()
    compare(ctx, ref, 1e-12, True)
    if k >= 9:
        assert np.abs(np.tril(ref.Tk(), -1)).max() > 1e-9  # T is far from I
    v = W.normal(9, k, n)
    assert ref.add(v) == 0
    ctx.qr_add(to_dev(v))
    compare(ctx, ref, 1e-10, True)
    assert ctx.sync_counts()[1] == 0


@pytest.mark.parametrize("form", FORMS, ids=IDS)
@pytest.mark.parametrize("m", [1, 3, 10, 17])
@pytest.mark.parametrize("fuse_rhs", [False, True])
def test_aa_small_matches_oracle(form, m, fuse_rhs):
    """3D nonlinear map on a 21^3 grid and the 1D Poisson map, 20 iterations
    (the window recycles from iteration m + 1), grid-wide passes; with
    fuse_rhs, c = Q^T f_i from the QRAdd's reduction (the lagged DCGS-2 forms
    it from the same single reduction)."""
    device()
    from paper_2110_09667_amd import aa
    variant, lf, of = form
    flags = lf | (aa.FUSE_RHS if fuse_rhs else 0)
    for prob in (W.nonlinear3d(s=21, seed=6), W.poisson1d()):
        iters = 20
        xs_ref, st, _ = O.run_aa(lambda u: O.G_stencil(prob, u), np.zeros(prob.n), m, variant,
                                 iters, flags=of)
        xs, ctx = gpu_aa_run(prob, m, variant, iters, flags=flags)
        worst = max(max(rel(xs[i], xs_ref[i]), rel_inf(xs[i], xs_ref[i]))
                    for i in range(1, iters + 2))
        assert worst <= 1e-10, (prob.n, worst)
        info = ctx.info()
        assert info.status == 0
        add, dele, rhs = ctx.sync_counts()
        assert dele == 0  # neither form reduces in QRDelete
        if variant == "dcgs2_lag":
            assert add == iters  # one reduction per add
        else:  # ICWY: 2 per add into a non-empty window (m = 1 never has one)
            assert add == (iters if m == 1 else 1 + 2 * (iters - 1))
        assert rhs == (1 if fuse_rhs and m > 1 else iters), rhs


@pytest.mark.parametrize("form", FORMS, ids=IDS)
@pytest.mark.parametrize("m", [20, 50])
def test_recycled_window_matches_oracle(form, m):
    """48^3, m + 12 iterations (12 recycled): the first 20 iterations to
    1e-10, the rest to max(1e-10, 100 eps kappa_max) as for Algs. 3-6."""
    device()
    variant, lf, of = form
    prob = W.nonlinear3d(s=48, seed=6)
    iters = m + 12
    xs_ref, kappas, _ = oracle_trajectory(O, prob, m, variant, iters, flags=of)
    xs, ctx = gpu_aa_run(prob, m, variant, iters, flags=lf)
    assert ctx.info().status == 0
    kmax, worst20 = 1.0, 0.0
    for i in range(1, iters + 2):
        kmax = max(kmax, kappas[i])
        d = max(rel(xs[i], xs_ref[i]), rel_inf(xs[i], xs_ref[i]))
        tol = 1e-10 if i <= 20 else max(1e-10, 100 * EPS * kmax)
        assert d <= tol, (i, d, kmax)
        if i <= 20:
            worst20 = max(worst20, d)
    print(f"\n{variant} flags={lf} m={m}: first 20 {worst20:.2e}, kappa_max {kmax:.2e}")


@pytest.mark.parametrize("form", FORMS, ids=IDS)
def test_full_size_matches_oracle(form):
    """256^3 (n = 16,777,216), m = 5, 20 iterations."""
    device()
    variant, lf, of = form
    prob = W.nonlinear3d()
    iters = 20
    xs_ref, _, _ = O.run_aa(lambda u: O.G_stencil(prob, u), np.zeros(prob.n), 5, variant, iters,
                            flags=of)
    xs, ctx = gpu_aa_run(prob, 5, variant, iters, flags=lf)
    assert ctx.info().status == 0
    worst = max(max(rel(xs[i], xs_ref[i]), rel_inf(xs[i], xs_ref[i])) for i in range(1, iters + 2))
    assert worst <= 1e-10, worst
    print(f"\nfull size {variant} flags={lf}: {worst:.2e}")


def test_new_forms_refused_where_unsupported():
    device()
    import torch
    from paper_2110_09667_amd import aa
    probs = [W.batch_problem(i) for i in W.batch_table(2, first_seed=5, s_lo=8, s_hi=12)]
    with pytest.raises(aa.AAError):
        aa.AABatch(probs, [3, 3], "icwy", flags=aa.ICWY_T_TRANSFORM, tol=0.0, max_iter=10)
    with pytest.raises(aa.AAError):
        aa.AABatch(probs, [3, 3], "dcgs2_lag", tol=0.0, max_iter=10)
    # a breakdown of the lagged form is latched: a column already in the span
    ctx = aa.AAContext(1, 3, "dcgs2_lag", aa.QR_ONLY)
    ctx.qr_add(torch.tensor([3.0], dtype=torch.float64, device="cuda"))
    ctx.qr_add(torch.tensor([-2.0], dtype=torch.float64, device="cuda"))
    assert ctx.info().status == -3
