"""CPU oracle of the learned mixing-weight network (TEST INFRASTRUCTURE ONLY).

The network reads quantities of the windowed QR that do not depend on n --
the upper triangle of R (padded to a 20 x 20 window, 210 values) and
c = Q^T f_i (20 values), both divided by ||f_i||_2, since gamma = R^{-1} c is
unchanged by a common scale -- and proposes a correction to the AA mixing
weights gamma (20 values, masked to the m_i columns in use) and a damping
beta = sigmoid(o_20).  Architecture 230 -> 256 -> 256 -> 256 -> 21 with GELU
(the erf form), BF16 operands with FP32 accumulation, FP32 master weights.

This module computes the same network in FP64 but rounds to BF16
(round-to-nearest-even) exactly where the GPU kernels do: the input features,
the weights and the hidden activations entering each product, and the
upstream gradients entering the backward products.  With ``bf16=False`` it is
the plain FP64 network, pinned against central finite differences.

Padding: the first layer's input dimension is stored as 256 (features 230..255
are zero) and the last layer's output as 64 (outputs 21..63 are zero); padded
weights start at zero and receive zero gradients.
"""
from __future__ import annotations

import math

import numpy as np

WIN = 20                      # window the features are padded to
NF = WIN * (WIN + 1) // 2 + WIN   # 210 + 20 = 230 input features
NIN, NH, NOUT = 256, 256, 64  # padded layer widths
NO = WIN + 1                  # 21 live outputs: delta gamma (20) and beta logit
DIMS = [(NIN, NH), (NH, NH), (NH, NH), (NH, NOUT)]
BETA_BIAS = 4.0               # sigmoid(4) ~ 0.982: an untrained net is ~plain AA


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to float32 (as the GPU holds it)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    nan = np.isnan(f)
    r = (r << np.uint64(16)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def _erf(x):
    from scipy.special import erf
    return erf(x)


def features(R: np.ndarray, c: np.ndarray, fnorm: float) -> np.ndarray:
    """Feature vector of one AA state: upper triangle of R (row-major over
    a <= b < 20, zero outside the m_i x m_i block), then c, scaled by 1/||f||."""
    mi = R.shape[0]
    out = np.zeros(NF)
    p = 0
    for a in range(WIN):
        for b in range(a, WIN):
            if b < mi:
                out[p] = R[a, b]
            p += 1
    out[p:p + mi] = c[:mi]
    return out / fnorm


def forward(params, X: np.ndarray, bf16_casts: bool = True):
    """params: list of (W [in x out], b [out]) float arrays (padded shapes).
    X: [B x 230] features.  Returns (out [B x 64], cache for backward)."""
    rnd = bf16 if bf16_casts else (lambda a: np.asarray(a, dtype=np.float64))
    B = X.shape[0]
    h = np.zeros((B, NIN))
    h[:, :NF] = X
    h = rnd(h)
    cache = []
    for l, (W, b) in enumerate(params):
        z = h @ rnd(W) + b
        cache.append((h, z))
        if l < len(params) - 1:
            h = rnd(gelu(z))
        else:
            out = z
    return out, cache


def backward(params, cache, dout: np.ndarray, bf16_casts: bool = True):
    """dout: [B x 64] gradient of the loss w.r.t. the network output.
    Returns [(dW, db)] per layer (FP64)."""
    rnd = bf16 if bf16_casts else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(params)
    dz = np.asarray(dout, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h, z = cache[l]
        dzr = rnd(dz)
        grads[l] = (h.T @ dzr, dz.sum(axis=0))
        if l > 0:
            dh = dzr @ rnd(W).T
            dz = dh * gelu_grad(cache[l - 1][1])
    return grads


def decode(out: np.ndarray, mi: np.ndarray):
    """delta gamma (masked to the first m_i entries) and beta = sigmoid(o_20)."""
    dg = out[:, :WIN].copy()
    for r, m in enumerate(mi):
        dg[r, m:] = 0.0
    beta = 1.0 / (1.0 + np.exp(-out[:, WIN]))
    return dg, beta


def adam(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on FP32 master weights (in place); state: list of (m, v)."""
    new = []
    for (W, b), (gW, gb), (mv) in zip(params, grads, state):
        out = []
        for P, G, (M, V) in ((W, gW, mv[0]), (b, gb, mv[1])):
            M[...] = b1 * M + (1 - b1) * G
            V[...] = b2 * V + (1 - b2) * G * G
            mh = M / (1 - b1 ** t)
            vh = V / (1 - b2 ** t)
            P -= lr * mh / (np.sqrt(vh) + eps)
            out.append(P)
        new.append(tuple(out))
    return new
