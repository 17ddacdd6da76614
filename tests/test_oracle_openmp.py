"""The OpenMP build of the oracle (the CPU baseline) computes bitwise what the
single-threaded build computes, for any thread count: dot products sum fixed
row blocks in block order, and every other row loop is elementwise.  Run in a
child process so that switching libraries does not touch the other tests."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, %r)
import aa_workloads as W, oracle as O
prob = W.nonlinear3d(s=48, seed=6)   # n = 110,592: two dot-product blocks
def run():
    out = []
    for v in ("mgs", "icwy", "dcgs2_lag"):
        xs, st, _ = O.run_aa(lambda u: O.G_stencil(prob, u), np.zeros(prob.n), 4, v, 9)
        out.append(np.stack(xs))
        out.append(st.Rk())
    return out
ref = run()
for t in (1, 3, 8):
    got_t = O.use_openmp(t)
    got = run()
    assert all(np.array_equal(a, b) for a, b in zip(ref, got)), t
print("ok", got_t)
""" % ROOT


def test_openmp_build_is_bitwise_single_threaded():
    import oracle
    oracle.build(force=False)
    r = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.startswith("ok")
