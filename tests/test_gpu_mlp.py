"""The BF16 MFMA network kernels against the CPU oracle that emulates BF16
round-to-nearest-even at the same points (forward, backward, Adam), plus the
initialization invariants.  Parameters and inputs come from the shared seeded
generator, uploaded to both sides."""
import numpy as np
import pytest

import aa_workloads as W
from gpu_util import device
from oracle import mlp as M

pytestmark = pytest.mark.gpu


def packed_random(seed, scale=0.25):
    """Seeded FP32 parameters in the packed layout, padding zero."""
    parts, params = [], []
    for l, (i, o) in enumerate(M.DIMS):
        Wl = (W.normal(seed, 2 * l, i * o) * scale / np.sqrt(i)).reshape(i, o)
        bl = W.normal(seed, 2 * l + 1, o) * 0.1
        if l == 0:
            Wl[M.NF:, :] = 0.0
        if l == len(M.DIMS) - 1:
            Wl[:, M.NO:] = 0.0
            bl[M.NO:] = 0.0
        Wl = Wl.astype(np.float32)
        bl = bl.astype(np.float32)
        params.append((Wl.astype(np.float64), bl.astype(np.float64)))
        parts += [Wl.ravel(), bl]
    return np.concatenate(parts), params


def unpack(vec):
    out, o = [], 0
    for (i, oo) in M.DIMS:
        Wl = vec[o:o + i * oo].reshape(i, oo)
        o += i * oo
        bl = vec[o:o + oo]
        o += oo
        out.append((Wl, bl))
    return out


@pytest.mark.parametrize("batch", [1, 37, 300])
def test_forward_matches_oracle(batch):
    import torch
    device()
    from paper_2110_09667_amd import aa
    net = aa.AAMlp(512)
    flat, params = packed_random(11)
    net.set_params(flat)
    X = (W.normal(12, 0, batch * M.NF).reshape(batch, M.NF)).astype(np.float32)
    xd = torch.from_numpy(X).cuda()
    out = torch.empty(batch, M.NO, dtype=torch.float32, device="cuda")
    net.forward(xd, out)
    ref, _ = M.forward(params, X.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    r = ref[:, :M.NO]
    assert np.linalg.norm(got - r) <= 1e-3 * np.linalg.norm(r)
    big = np.abs(r) > 1e-2 * np.abs(r).max()
    assert np.all(np.abs(got - r)[big] <= 1e-2 * np.abs(r)[big])


def test_backward_matches_oracle():
    import torch
    device()
    from paper_2110_09667_amd import aa
    batch = 133
    net = aa.AAMlp(256)
    flat, params = packed_random(21)
    net.set_params(flat)
    X = W.normal(22, 0, batch * M.NF).reshape(batch, M.NF).astype(np.float32)
    D = W.normal(23, 0, batch * M.NO).reshape(batch, M.NO).astype(np.float32)
    net.forward(torch.from_numpy(X).cuda())
    net.backward(torch.from_numpy(D).cuda())
    got = unpack(net.get_grads().astype(np.float64))
    _, cache = M.forward(params, X.astype(np.float64))
    dout = np.zeros((batch, M.NOUT))
    dout[:, :M.NO] = D
    ref = M.backward(params, cache, dout)
    for l in range(4):
        for a, b in ((got[l][0], ref[l][0]), (got[l][1], ref[l][1])):
            assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-30, l
    # padding receives no gradient
    assert np.all(got[0][0][M.NF:, :] == 0.0)
    assert np.all(got[3][0][:, M.NO:] == 0.0)


def test_init_gives_no_correction_and_beta_bias():
    import torch
    device()
    from paper_2110_09667_amd import aa
    net = aa.AAMlp(64, seed=5)
    X = torch.from_numpy(W.normal(1, 0, 64 * M.NF).reshape(64, M.NF).astype(np.float32)).cuda()
    out = torch.empty(64, M.NO, dtype=torch.float32, device="cuda")
    net.forward(X, out)
    o = out.cpu().numpy()
    assert np.all(o[:, :M.WIN] == 0.0)
    assert np.all(o[:, M.WIN] == np.float32(M.BETA_BIAS))
    p = unpack(net.get_params().astype(np.float64))
    assert np.all(p[0][0][M.NF:, :] == 0.0) and np.all(p[3][0] == 0.0)
    w = p[1][0]
    assert abs(w.std() * np.sqrt(256) / np.sqrt(2.0) - 1.0) < 0.05  # He scale


def test_adam_step_matches_oracle():
    import torch
    device()
    from paper_2110_09667_amd import aa
    batch = 64
    net = aa.AAMlp(batch)
    flat, params = packed_random(31)
    net.set_params(flat)
    X = W.normal(32, 0, batch * M.NF).reshape(batch, M.NF).astype(np.float32)
    D = W.normal(33, 0, batch * M.NO).reshape(batch, M.NO).astype(np.float32)
    net.forward(torch.from_numpy(X).cuda())
    net.backward(torch.from_numpy(D).cuda())
    g = unpack(net.get_grads().astype(np.float64))
    net.adam(lr=1e-2)
    new = unpack(net.get_params().astype(np.float64))
    state = [((np.zeros_like(Wl), np.zeros_like(Wl)), (np.zeros_like(bl), np.zeros_like(bl)))
             for Wl, bl in params]
    ref = M.adam([(Wl.copy(), bl.copy()) for Wl, bl in params], g, state, 1e-2, 1)
    for l in range(4):
        assert np.allclose(new[l][0], ref[l][0], rtol=1e-5, atol=1e-6)
        assert np.allclose(new[l][1], ref[l][1], rtol=1e-5, atol=1e-6)
    assert np.all(net.get_grads() == 0.0)
