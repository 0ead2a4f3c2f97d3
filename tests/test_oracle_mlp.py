"""Pins of the oracle's surrogate network: gradients by central finite
differences and by PyTorch CPU autograd (an independent implementation),
GELU against its integral definition, bfloat16 rounding against PyTorch."""
import numpy as np
import pytest
import torch
from scipy.integrate import quad

from oracle import mlp


def test_gelu_is_z_times_normal_cdf_and_grad_matches():
    z = np.linspace(-6, 6, 41)
    cdf = np.array([quad(lambda t: np.exp(-t * t / 2) / np.sqrt(2 * np.pi), -np.inf, v)[0] for v in z])
    np.testing.assert_allclose(mlp.gelu(z), z * cdf, atol=1e-10)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) + 0.05 * rng.standard_normal(mlp.NPARAM)
    X = rng.standard_normal((17, mlp.NIN))
    Y = rng.standard_normal((17, mlp.NOUT))
    _, g = mlp.backward(theta, X, Y)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(theta + e, X, Y) - mlp.loss(theta - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    rng = np.random.default_rng(1)
    theta = mlp.init_params(2)
    X = rng.standard_normal((33, mlp.NIN))
    Y = rng.standard_normal((33, mlp.NOUT))
    L, g = mlp.backward(theta, X, Y)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o, params = 0, {}
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        params[name] = t[o:o + n].reshape(shape)
        o += n
    x = torch.tensor(X)
    h = x
    for i in (1, 2, 3):
        h = torch.nn.functional.gelu(h @ params[f"W{i}"].T + params[f"b{i}"])
    y = h @ params["W4"].T + params["b4"]
    lt = ((y - torch.tensor(Y)) ** 2).mean()
    lt.backward()
    assert abs(lt.item() - L) < 1e-13
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(10000) * 10 ** rng.uniform(-5, 5, 10000)
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(a), ref)


def test_adam_step_matches_torch():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    t = torch.tensor(theta, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2)
    m = np.zeros(50)
    v = np.zeros(50)
    for k in range(1, 4):
        g = rng.standard_normal(50)
        t.grad = torch.tensor(g)
        opt.step()
        theta, m, v = mlp.adam_step(theta, m, v, g, k, 1e-2)
    np.testing.assert_allclose(theta, t.detach().numpy(), rtol=1e-12, atol=1e-14)
