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


def test_quantised_forward_matches_torch_bfloat16_casts():
    """An independent implementation of the quantised forward: PyTorch's
    own bfloat16 casts of the input, of every weight matrix and of every
    hidden activation, FP64 matrix products, FP64 biases (not rounded), its
    erf-form GELU."""
    rng = np.random.default_rng(12)
    theta = mlp.init_params(5)
    p = mlp.unpack(theta)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.3 * rng.standard_normal(p[k].shape)
    theta = mlp.pack(p)
    X = rng.standard_normal((257, mlp.NIN)) * 1.7
    q = lambda a: torch.tensor(a).to(torch.bfloat16).to(torch.float64)
    h = q(X)
    for i in (1, 2, 3):
        z = h @ q(p[f"W{i}"]).T + torch.tensor(p[f"b{i}"])
        h = torch.nn.functional.gelu(z).to(torch.bfloat16).to(torch.float64)
    ref = (h @ q(p["W4"]).T + torch.tensor(p["b4"])).numpy()
    got = mlp.quantised_forward(theta, X)
    # both accumulate in FP64; only the summation order and the two erf
    # implementations differ (a rounding flip of an activation moves an
    # output by ~2^-9 of one term, which no case here comes near)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    # the quantisation is visible: the exact forward differs by far more
    assert np.abs(mlp.forward(theta, X) - got).max() > 1e-4


def _bf16_scalar(x):
    """Round one float to bfloat16 by hand: to FP32 first, then keep the top
    16 bits, rounding the dropped 16 to nearest, ties to even."""
    import struct
    u = struct.unpack("<I", struct.pack("<f", x))[0]
    low, high = u & 0xFFFF, u >> 16
    if low > 0x8000 or (low == 0x8000 and (high & 1)):
        high += 1
    return struct.unpack("<f", struct.pack("<I", high << 16))[0]


def test_quantised_forward_one_unit_by_hand():
    """One active path through the network, evaluated by hand with scalar
    arithmetic: input x0 = 1/3, W1[0,0] = 3, b1[0] = -0.1, W2[0,0] = 0.7,
    b2[0] = -0.05, W3[0,0] = 1.3, b3[0] = 0.2, W4[k,0] = (0.9, -0.4, 2.1),
    b4 = (0.1, 0.02, 0.03); every other parameter and input is 0, so every
    other hidden unit is GELU(0) = 0.  bfloat16 of 1/3 is 0x3EAB = 0.333984375
    (the dropped half 0xAAAB rounds up).  The values are chosen so that the
    two plausible slips, leaving the input unrounded or rounding the biases,
    each move an output by more than 1e-3."""
    from math import erf, sqrt
    W1, b1, W2, b2, W3, b3 = 3.0, -0.1, 0.7, -0.05, 1.3, 0.2
    W4, b4 = (0.9, -0.4, 2.1), (0.1, 0.02, 0.03)
    theta = np.zeros(mlp.NPARAM)
    p = mlp.unpack(theta)
    p["W1"][0, 0], p["b1"][0] = W1, b1
    p["W2"][0, 0], p["b2"][0] = W2, b2
    p["W3"][0, 0], p["b3"][0] = W3, b3
    p["W4"][:, 0] = W4
    p["b4"][:] = b4
    theta = mlp.pack(p)
    X = np.zeros((1, mlp.NIN))
    X[0, 0] = 1.0 / 3.0
    assert _bf16_scalar(1.0 / 3.0) == 0.333984375
    q = _bf16_scalar
    g = lambda z: 0.5 * z * (1.0 + erf(z / sqrt(2.0)))

    def by_hand(round_input=True, round_bias=False):
        x = q(1.0 / 3.0) if round_input else 1.0 / 3.0
        bb = q if round_bias else (lambda v: v)
        h1 = q(g(q(W1) * x + bb(b1)))
        h2 = q(g(q(W2) * h1 + bb(b2)))
        h3 = q(g(q(W3) * h2 + bb(b3)))
        return np.array([q(w) * h3 + bb(c) for w, c in zip(W4, b4)])

    got = mlp.quantised_forward(theta, X)[0]
    np.testing.assert_allclose(got, by_hand(), rtol=0, atol=1e-15)
    # the planted slips land far outside that tolerance
    assert np.abs(by_hand(round_input=False) - got).max() > 1e-3
    assert np.abs(by_hand(round_bias=True) - got).max() > 1e-3


def test_quantised_backward_without_rounding_is_the_gradient():
    rng = np.random.default_rng(6)
    theta = mlp.init_params(8) + 0.05 * rng.standard_normal(mlp.NPARAM)
    X = rng.standard_normal((40, mlp.NIN))
    Y = rng.standard_normal((40, mlp.NOUT))
    L, g = mlp.backward(theta, X, Y)
    Lq, gq = mlp.quantised_backward(theta, X, Y, rnd=lambda a: a)
    assert abs(L - Lq) <= 1e-15 * L
    np.testing.assert_allclose(gq, g, rtol=1e-12, atol=1e-16)
    # with bfloat16 operands: a few roundings of 2^-9 per term, normwise
    _, gb = mlp.quantised_backward(theta, X, Y)
    assert np.linalg.norm(gb - g) <= 2e-2 * np.linalg.norm(g)
    assert np.linalg.norm(gb - g) > 1e-5 * np.linalg.norm(g)


def test_quantised_backward_one_unit_by_hand():
    """The one-path network of the forward case with target Y, its gradient
    by hand: dL/dy = 2 (y - Y)/3 rounded; W4's column 0 and b4 from it; then
    dz3 = rnd(a3 GELU'(z3)) with a3 = sum_o dy_o rnd(W4[o,0]), and so on down
    to W1[0,0] = dz1 rnd(x0).  Every other element is 0 (the other hidden
    units have z = 0 and receive no error).  Leaving dz unrounded, or the
    GELU' factor out, moves elements by more than 1e-4 relative."""
    from math import erf, exp, pi, sqrt
    W1, b1, W2, b2, W3, b3 = 3.0, -0.1, 0.7, -0.05, 1.3, 0.2
    W4, b4 = (0.9, -0.4, 2.1), (0.1, 0.02, 0.03)
    Yt = (0.5, -0.3, 0.2)
    theta = np.zeros(mlp.NPARAM)
    p = mlp.unpack(theta)
    p["W1"][0, 0], p["b1"][0] = W1, b1
    p["W2"][0, 0], p["b2"][0] = W2, b2
    p["W3"][0, 0], p["b3"][0] = W3, b3
    p["W4"][:, 0] = W4
    p["b4"][:] = b4
    theta = mlp.pack(p)
    X = np.zeros((1, mlp.NIN))
    X[0, 0] = 1.0 / 3.0
    q = _bf16_scalar
    g = lambda z: 0.5 * z * (1.0 + erf(z / sqrt(2.0)))
    gp = lambda z: 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2 * pi)

    def by_hand(round_dz=True, gelu_factor=True):
        r = q if round_dz else (lambda v: v)
        f = gp if gelu_factor else (lambda z: 1.0)
        x = q(1.0 / 3.0)
        z1 = q(W1) * x + b1
        h1 = q(g(z1))
        z2 = q(W2) * h1 + b2
        h2 = q(g(z2))
        z3 = q(W3) * h2 + b3
        h3 = q(g(z3))
        y = [q(w) * h3 + c for w, c in zip(W4, b4)]
        dy = [r(2.0 * (yo - to) / 3.0) for yo, to in zip(y, Yt)]
        out = {"W4": [d * h3 for d in dy], "b4": dy}
        dz3 = r(sum(d * q(w) for d, w in zip(dy, W4)) * f(z3))
        dz2 = r(dz3 * q(W3) * f(z2))
        dz1 = r(dz2 * q(W2) * f(z1))
        out.update(W3=dz3 * h2, b3=dz3, W2=dz2 * h1, b2=dz2, W1=dz1 * x, b1=dz1)
        return out

    want = by_hand()
    L, gq = mlp.quantised_backward(theta, X, np.array([Yt]))
    G = mlp.unpack(gq)
    for k in ("W4", "b4"):
        got = G[k][:, 0] if k == "W4" else G[k]
        np.testing.assert_allclose(got, want[k], rtol=1e-15, atol=0)
    for i in (1, 2, 3):
        assert abs(G[f"W{i}"][0, 0] - want[f"W{i}"]) <= 1e-15 * abs(want[f"W{i}"])
        assert abs(G[f"b{i}"][0] - want[f"b{i}"]) <= 1e-15 * abs(want[f"b{i}"])
    mask = np.ones(mlp.NPARAM, bool)
    off = 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        blk = np.zeros(shape, bool)
        if name == "W4":
            blk[:, 0] = True
        elif name == "b4":
            blk[:] = True
        elif name.startswith("W"):
            blk[0, 0] = True
        else:
            blk[0] = True
        mask[off:off + n] = ~blk.ravel()
        off += n
    assert not gq[mask].any()
    # planted slips move the deeper elements well beyond the tolerance
    for slip in (by_hand(round_dz=False), by_hand(gelu_factor=False)):
        assert max(abs(slip[k] - want[k]) / abs(want[k]) for k in ("W1", "W2", "b1")) > 1e-4
