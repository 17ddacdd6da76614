"""Pins of the CPU network oracle: BF16 rounding against hand-computed ties,
the FP64 backward against central finite differences, the feature map
against its definition, and the untrained network's output (an exact zero
correction and beta = sigmoid(4))."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_round_to_nearest_even():
    # bf16 keeps 7 fraction bits: spacing 2^-7 on [1, 2)
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7,
                  -1.0 - 3 * 2.0 ** -8, 3.0e38, 1e-40, 0.0])
    got = mlp.bf16(x)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # tie -> even mantissa (0)
    assert got[2] == 1.0 + 2 * 2.0 ** -7      # tie -> even mantissa (2)
    assert got[3] == 1.0 + 2.0 ** -7          # exactly representable
    assert got[4] == -(1.0 + 2 * 2.0 ** -7)
    assert np.isfinite(got[5]) or got[5] == np.inf
    assert got[7] == 0.0
    r = np.random.default_rng(0).standard_normal(10000)
    e = np.abs(mlp.bf16(r) - r) / np.abs(r)
    assert e.max() <= 2.0 ** -8 * (1 + 1e-9)  # half an ulp of 8 significant bits


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    params = []
    for (i, o) in mlp.DIMS:
        W = rng.standard_normal((i, o)) * scale / np.sqrt(i)
        b = rng.standard_normal(o) * 0.1
        params.append((W, b))
    W0, b0 = params[0]
    W0[mlp.NF:, :] = 0.0
    W3, b3 = params[3]
    W3[:, mlp.NO:] = 0.0
    b3[mlp.NO:] = 0.0
    return params


def loss_fn(params, X, T):
    out, cache = mlp.forward(params, X, bf16_casts=False)
    return 0.5 * np.sum((out[:, :mlp.NO] - T) ** 2), out, cache


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    params = random_params(2)
    X = rng.standard_normal((5, mlp.NF))
    T = rng.standard_normal((5, mlp.NO))
    L, out, cache = loss_fn(params, X, T)
    dout = np.zeros_like(out)
    dout[:, :mlp.NO] = out[:, :mlp.NO] - T
    grads = mlp.backward(params, cache, dout, bf16_casts=False)
    h = 1e-6
    for l, (i, j) in [(0, (3, 7)), (0, (229, 100)), (1, (5, 5)), (2, (200, 17)),
                      (3, (10, 20)), (3, (255, 0))]:
        W = params[l][0]
        old = W[i, j]
        W[i, j] = old + h
        Lp = loss_fn(params, X, T)[0]
        W[i, j] = old - h
        Lm = loss_fn(params, X, T)[0]
        W[i, j] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(grads[l][0][i, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, i, j)
    for l, j in [(0, 3), (2, 250), (3, 20)]:
        b = params[l][1]
        old = b[j]
        b[j] = old + h
        Lp = loss_fn(params, X, T)[0]
        b[j] = old - h
        Lm = loss_fn(params, X, T)[0]
        b[j] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(grads[l][1][j] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, j)


def test_padded_weights_get_zero_gradient():
    rng = np.random.default_rng(3)
    params = random_params(4)
    X = rng.standard_normal((7, mlp.NF))
    out, cache = mlp.forward(params, X)
    dout = np.zeros_like(out)
    dout[:, :mlp.NO] = rng.standard_normal((7, mlp.NO))
    grads = mlp.backward(params, cache, dout)
    assert np.all(grads[0][0][mlp.NF:, :] == 0.0)
    assert np.all(grads[3][0][:, mlp.NO:] == 0.0)
    assert np.all(grads[3][1][mlp.NO:] == 0.0)


def test_bf16_forward_close_to_fp64():
    rng = np.random.default_rng(5)
    params = random_params(6)
    X = rng.standard_normal((9, mlp.NF))
    a, _ = mlp.forward(params, X, bf16_casts=True)
    b, _ = mlp.forward(params, X, bf16_casts=False)
    assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b)


def test_features_definition():
    rng = np.random.default_rng(7)
    mi = 4
    R = np.triu(rng.standard_normal((mi, mi)))
    c = rng.standard_normal(mi)
    f = mlp.features(R, c, 2.0)
    assert f.shape == (mlp.NF,)
    # row 0 of the padded upper triangle occupies entries 0..19
    assert np.allclose(f[:mi], R[0, :] / 2.0) and np.all(f[mi:20] == 0.0)
    # row 1 starts at 20 and holds R[1, 1:20]
    assert np.allclose(f[20:20 + mi - 1], R[1, 1:] / 2.0)
    assert np.allclose(f[210:210 + mi], c / 2.0) and np.all(f[210 + mi:] == 0.0)
    assert np.count_nonzero(f) == mi * (mi + 1) // 2 + mi


def test_decode_masks_and_sigmoid():
    out = np.zeros((2, mlp.NOUT))
    out[:, :mlp.WIN] = 1.0
    out[0, mlp.WIN] = mlp.BETA_BIAS
    dg, beta = mlp.decode(out, np.array([3, 20]))
    assert np.all(dg[0, :3] == 1.0) and np.all(dg[0, 3:] == 0.0) and np.all(dg[1] == 1.0)
    assert abs(beta[0] - 1 / (1 + np.exp(-4.0))) < 1e-15 and beta[1] == 0.5


def test_gelu_fixed_values_and_odd_part():
    """GELU(z) = z * Phi(z), Phi the standard normal CDF (erf form, no tanh
    approximation).  Phi at 0.5, 1, 2 are textbook table values; Phi is also
    recomputed here by integrating the normal density (an independent route);
    and Phi(z) + Phi(-z) = 1 gives GELU(z) - GELU(-z) = z."""
    from scipy.integrate import quad
    table = {0.5: 0.6914624612740131, 1.0: 0.8413447460685429, 2.0: 0.9772498680518208}
    for z, phi in table.items():
        assert abs(mlp.gelu(np.array([z]))[0] - z * phi) <= 1e-15 * z
        dens = quad(lambda t: np.exp(-0.5 * t * t) / np.sqrt(2 * np.pi), -np.inf, z,
                    epsabs=1e-15, epsrel=1e-14)[0]
        assert abs(dens - phi) <= 1e-13
    # the tanh approximation is off by ~1.5e-4 at z = 1: a 1e-12 pin rejects it
    z = np.linspace(-6.0, 6.0, 241)
    assert np.max(np.abs(mlp.gelu(z) - mlp.gelu(-z) - z)) <= 1e-14
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # tails: GELU(z) -> z for large z, -> 0 for very negative z
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) <= 1e-15 * 10
    assert abs(mlp.gelu(np.array([-10.0]))[0]) <= 1e-20


def test_adam_first_two_steps_closed_form():
    """Adam (Kingma and Ba, Alg. 1): with bias correction the first step moves
    every weight by -lr g / (|g| + eps), whatever beta1 and beta2 are; the
    second step's moments are worked out by hand below, which tells a swap of
    beta1 and beta2 or a missing bias correction from the right update."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    g1 = np.array([[0.5, -2.0], [1e-3, 0.0]])
    g2 = np.array([[-1.5, 4.0], [2e-3, 3.0]])
    W = np.array([[1.0, 2.0], [3.0, 4.0]])
    b = np.array([0.25, -0.25])
    gb1, gb2 = np.array([0.1, -0.2]), np.array([0.3, 0.05])
    params = [(W.copy(), b.copy())]
    # per layer: (first, second) moments of W, then of b
    state = [((np.zeros_like(W), np.zeros_like(W)), (np.zeros_like(b), np.zeros_like(b)))]
    params = mlp.adam(params, [(g1, gb1)], [state[0]], lr, 1, b1, b2, eps)
    W1 = W - lr * g1 / (np.abs(g1) + eps)
    bb1 = b - lr * gb1 / (np.abs(gb1) + eps)
    assert np.allclose(params[0][0], W1, rtol=0, atol=1e-15)
    assert np.allclose(params[0][1], bb1, rtol=0, atol=1e-15)
    params = mlp.adam(params, [(g2, gb2)], [state[0]], lr, 2, b1, b2, eps)
    # moments after two steps: m = 0.09 g1 + 0.1 g2, v = 0.000999 g1^2 + 0.001 g2^2;
    # bias corrections 1 - 0.9^2 = 0.19 and 1 - 0.999^2 = 0.001999
    for P0, ga, gb_, P in ((W1, g1, g2, params[0][0]), (bb1, gb1, gb2, params[0][1])):
        mh = (0.09 * ga + 0.1 * gb_) / 0.19
        vh = (0.000999 * ga * ga + 0.001 * gb_ * gb_) / 0.001999
        assert np.allclose(P, P0 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-14)
