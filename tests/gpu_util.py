"""Helpers of the GPU tests: device checks and the HIP-path drivers.

The HIP side is driven only through the C ABI (``paper_2110_09667_amd.aa``);
the expected values come only from ``oracle`` on the same seeded inputs.
"""
import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_09667_amd import aa
    aa.lib()  # raises if the HIP library is missing: no silent fallback
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def gpu_aa_run(prob, m, variant, iters, flags=0, x0=None, record=True, fused=None):
    """Run AA on the GPU with the library's stencil map; returns the iterates
    x_0..x_{iters+1} (numpy) and the context.  fused: None = library default
    (one-workgroup step for small n), True = always, False = never."""
    import torch
    from paper_2110_09667_amd import aa
    dev = torch.device("cuda:0")
    n = prob.n
    f_d = to_dev(prob.f)
    ctx = aa.AAContext(n, m, variant, flags)
    if fused is not None:
        ctx.set_fused_threshold(1 << 40 if fused else 0)
    x = to_dev(np.zeros(n) if x0 is None else x0)
    g = torch.empty_like(x)
    xs = [x.cpu().numpy()]
    for _ in range(iters + 1):
        aa.aa_problem_apply(prob.d, prob.s, prob.h, prob.omega, prob.c, f_d, x, g)
        ctx.step(x, g, x)
        if record:
            xs.append(x.cpu().numpy())
    torch.cuda.synchronize(dev)
    return xs, ctx


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_inf(a, b):
    """Element-wise comparison as one number: max |a - b| / max |b|."""
    mb = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)


def oracle_trajectory(O, prob, m, variant, iters, flags=0):
    """The oracle's iterates x_0..x_{iters+1} and, per step, kappa_2(R) of the
    factorization the step solved with (1 before the first QR exists)."""
    st = O.AA(prob.n, m, variant, flags)
    x = np.zeros(prob.n)
    xs, kappas = [x.copy()], [1.0]
    for _ in range(iters + 1):
        g = O.G_stencil(prob, x)
        x = st.step(x, g)
        xs.append(x.copy())
        kappas.append(np.linalg.cond(st.Rk()) if st.k > 0 else 1.0)
    return xs, kappas, st
