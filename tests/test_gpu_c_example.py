"""The C ABI driven from plain C (``paper_2110_09667_amd/examples/aa_example``,
built by ``__graft_entry__.build()``): the program allocates its own device
buffers, runs AA on the 1D Poisson map and writes the final iterate; it must
equal, bit for bit, the same run through the Python binding (same kernels,
same order) -- on the one-workgroup path and on the grid-wide passes."""
import os
import subprocess

import numpy as np
import pytest

import aa_workloads as W
from gpu_util import device

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_2110_09667_amd", "examples", "aa_example")


@pytest.mark.parametrize("n,m,variant", [(4096, 5, 3), (65536, 8, 1), (65536, 8, 0)])
def test_c_example_matches_binding(tmp_path, n, m, variant):
    import torch
    device()
    from paper_2110_09667_amd import aa
    assert os.path.exists(EXAMPLE), "C example not built (run __graft_entry__.build())"
    prob = W.poisson1d(n=n)
    iters = 30
    out = tmp_path / "x.bin"
    r = subprocess.run([EXAMPLE, str(out), str(n), str(m), str(variant), str(iters),
                        repr(prob.omega), repr(prob.h)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "iteration 30" in r.stdout
    x_c = np.fromfile(out, dtype=np.float64)
    ctx = aa.AAContext(n, m, variant)
    f_d = torch.from_numpy(prob.f).cuda()
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x)
    for _ in range(iters + 1):
        aa.aa_problem_apply(1, n, prob.h, prob.omega, 0.0, f_d, x, g)
        ctx.step(x, g, x)
    assert np.array_equal(x_c, x.cpu().numpy())
