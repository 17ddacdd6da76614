"""aa_qr_solve_noalloc (the context-free solve that allocates nothing: its
partials live in a fixed device array) against aa_qr_solve on the same
factorization, through the C ABI: two calls in a row, the second with a
smaller n and k, so the second reuses the array the first left behind."""
import numpy as np
import pytest

from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu


def graded(n, m, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (U * np.logspace(0, -np.log10(kappa), m)) @ V.T


def solve_both(n, k, variant, seed):
    import torch
    from paper_2110_09667_amd import aa
    ctx = aa.AAContext(n, k, variant, aa.QR_ONLY)
    F = graded(n, k, 1e3, seed)
    for t in range(k):
        ctx.qr_add(to_dev(F[:, t]))
    f = to_dev(np.random.default_rng(seed + 1).standard_normal(n))
    g_ctx = torch.empty(k, dtype=torch.float64, device="cuda")
    ctx.qr_solve(f, g_ctx)
    Q, ldq = aa.aa_qr_basis(ctx.ctx)
    # R column-major with leading dimension k: the row-major storage of R^T
    R = torch.from_numpy(np.ascontiguousarray(ctx.get_qr()[0].T)).cuda()
    g_na = torch.full((k,), np.nan, dtype=torch.float64, device="cuda")
    lib = aa.lib()
    st = lib.aa_qr_solve_noalloc(Q, ldq, n, k, R.data_ptr(), k, f.data_ptr(), g_na.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    torch.cuda.synchronize()
    a, b = g_ctx.cpu().numpy(), g_na.cpu().numpy()
    ctx.close()
    return a, b


@pytest.mark.parametrize("variant", ["icwy", "mgs"])
def test_noalloc_solve_matches_context_solve(variant):
    device()
    for (n, k, seed) in ((1024 * 1024 + 777, 64, 5), (50_001, 7, 9)):
        a, b = solve_both(n, k, variant, seed)
        # the same kernels and grid: the same reduction order
        assert np.all(np.isfinite(b)) and rel(b, a) <= 1e-14, (n, k, rel(b, a))
        print(f"\nnoalloc {variant} n={n} k={k}: rel diff {rel(b, a):.1e} "
              f"(bitwise equal: {np.array_equal(a, b)})")


def test_noalloc_rejects_bad_sizes():
    device()
    from paper_2110_09667_amd import aa
    lib = aa.lib()
    # k beyond the fixed array's reach, k = 0, ldr < k, ldq < n: refused before any work
    assert lib.aa_qr_solve_noalloc(8, 100, 100, 65, 16, 65, 24, 32, None) == -1
    assert lib.aa_qr_solve_noalloc(8, 100, 100, 0, 16, 4, 24, 32, None) == -1
    assert lib.aa_qr_solve_noalloc(8, 100, 100, 5, 16, 4, 24, 32, None) == -1
    assert lib.aa_qr_solve_noalloc(8, 99, 100, 5, 16, 5, 24, 32, None) == -1
    assert lib.aa_qr_solve_noalloc(None, 100, 100, 5, 16, 5, 24, 32, None) == -1
