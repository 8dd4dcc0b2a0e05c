"""Pins of the surrogate MLP oracle: bfloat16 rounding against torch's own
conversion, GELU against known values of the normal CDF and its derivative
by finite differences, the backward pass against central differences of the
loss, Adam's first step against its closed form, and the parameter count."""
import math

import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


def _params(seed, layers=(5, 16, 16, 4)):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(rng.uniform(-1, 1, (a, b)) * math.sqrt(6.0 / a), rng.normal(0, 0.1, b))
            for a, b in zip(layers[:-1], layers[1:])]


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.standard_normal(100000) * 10 ** rng.uniform(-5, 5, 100000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gelu_values_and_derivative():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # Phi(1) and Phi(-2) of the standard normal
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-2.0]))[0] - (-2.0 * 0.022750131948179195)) < 1e-15
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-9)


def test_backward_matches_finite_differences():
    P = _params(2)
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((7, 5))
    T = rng.standard_normal((7, 4))
    loss, g = mlp.backward(P, X, T, bf16_ops=False)
    h = 1e-6
    for l, (W, b) in enumerate(P):
        for arr, ga in ((W, g[l][0]), (b, g[l][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.mse(mlp.forward(P, X, False)[0], T)
                flat[idx] = old - h
                lm = mlp.mse(mlp.forward(P, X, False)[0], T)
                flat[idx] = old
                assert abs(ga.reshape(-1)[idx] - (lp - lm) / (2 * h)) < 1e-7


def test_adam_first_step_closed_form():
    """After one step with zero moments, m_hat = g and v_hat = g^2, so every
    parameter moves by lr * g / (|g| + eps)."""
    P = _params(4)
    g = [(np.full_like(W, 0.3), np.full_like(b, -2.0)) for W, b in P]
    newp, _, _ = mlp.adam_step(P, g, mlp.zeros_like(P), mlp.zeros_like(P), 1, 1e-3)
    for (W, b), (W1, b1) in zip(P, newp):
        np.testing.assert_allclose(W - W1, 1e-3 * 0.3 / (0.3 + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(b - b1, -1e-3 * 2.0 / (2.0 + 1e-8), rtol=1e-12)


def test_parameter_count():
    assert mlp.n_params() == 207393


def test_bf16_network_close_to_fp64_network():
    """Rounding the GEMM operands to bfloat16 perturbs the outputs by about
    the bfloat16 unit roundoff (2^-8), not more."""
    P = _params(5, mlp.LAYERS)
    rng = np.random.Generator(np.random.PCG64(6))
    X = rng.standard_normal((64, 5))
    y16 = mlp.forward(P, X, True)[0]
    y64 = mlp.forward(P, X, False)[0]
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 2e-2
