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


def _torch_forward(P, X, bf16_ops):
    """Independent float64 reference of the network: torch's F.linear per
    layer (y = x W^T + b with W stored out x in), the exact-erf GELU on the
    hidden layers only, a linear output layer.  With bf16_ops the GEMM
    operands go through torch's own bfloat16 conversion."""
    import torch.nn.functional as F

    def op(a):
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        return t.float().to(torch.bfloat16).double() if bf16_ops else t

    h = torch.from_numpy(np.asarray(X, dtype=np.float64))
    for l, (W, b) in enumerate(P):
        h = F.linear(op(h.numpy()), op(np.ascontiguousarray(W.T)), torch.from_numpy(b))
        if l < len(P) - 1:
            h = F.gelu(h, approximate="none")
    return h.numpy()


@pytest.mark.parametrize("layers", [(5, 7, 3), (5, 256, 256, 256, 256, 33), (5, 40, 9, 40, 2)])
@pytest.mark.parametrize("bf16_ops", [False, True])
def test_forward_matches_torch_reference(layers, bf16_ops):
    """oracle mlp.forward against torch's layer primitives, non-square layers
    included (a transposed weight would not even multiply), to 1e-13."""
    P = _params(11, layers)
    rng = np.random.Generator(np.random.PCG64(12))
    X = rng.standard_normal((33, 5)) * 2.0
    got = mlp.forward(P, X, bf16_ops)[0]
    ref = _torch_forward(P, X, bf16_ops)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def _planted(kind):
    """Copies of mlp.forward with one plausible mistake each."""
    def fwd(params, X):
        h = np.asarray(X, dtype=np.float64)
        for l, (W, b) in enumerate(params):
            Wm = W.T if kind == "transposed" else W
            a = h @ Wm + (0.0 if kind == "no_bias" else b)
            if l < len(params) - 1 or kind == "gelu_on_output":
                h = mlp.gelu(a)
            else:
                h = a
        return h
    return fwd


@pytest.mark.parametrize("kind", ["gelu_on_output", "no_bias", "transposed"])
def test_forward_pin_catches_planted_mistakes(kind):
    """The torch reference separates the oracle's composition from each
    planted mistake (square layers, so the transposed weight still runs)."""
    P = _params(13, (5, 5, 5, 5))
    rng = np.random.Generator(np.random.PCG64(14))
    X = rng.standard_normal((17, 5))
    ref = _torch_forward(P, X, False)
    assert np.linalg.norm(mlp.forward(P, X, False)[0] - ref) <= 1e-13 * np.linalg.norm(ref)
    bad = _planted(kind)(P, X)
    assert np.linalg.norm(bad - ref) > 1e-3 * np.linalg.norm(ref)
