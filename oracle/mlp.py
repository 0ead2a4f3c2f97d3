"""FP64 reference of the ODE surrogate network (test infrastructure only).

Network 6 -> 64 -> 64 -> 64 -> 3, GELU (erf form, GELU(z) = z Phi(z)) after
each hidden layer, linear output.  Inputs are the per-voxel state the
intracellular ODEs see over one coupled step, (K, G1, G2, P, Vc, phi),
standardised; outputs the standardised update (dP, dVc, dphi).  Loss: mean
squared error over the batch and the three outputs.

Parameters are one flat vector in the order W1 (64x6), b1, W2 (64x64), b2,
W3 (64x64), b3, W4 (3x64), b4 - the same order the HIP library uses for its
gradient and Adam buffers.

``forward`` / ``backward`` are the plain definitions.  ``quantised_forward``
and ``quantised_backward`` define the network evaluated with bfloat16
operands: every operand of every matrix product (inputs, weights, hidden
activations, dL/dy and the back-propagated dZ) is rounded to bfloat16 (round
to nearest even), biases stay unrounded, products and sums are exact
(float64).  That is what matrix cores with bfloat16 inputs compute up to the
accumulation order, so GPU results can be compared with them at a tolerance
derived from that order alone.
"""
import numpy as np
from scipy.special import erf

NIN, NHID, NOUT = 6, 64, 3
SHAPES = [("W1", (NHID, NIN)), ("b1", (NHID,)), ("W2", (NHID, NHID)), ("b2", (NHID,)),
          ("W3", (NHID, NHID)), ("b3", (NHID,)), ("W4", (NOUT, NHID)), ("b4", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """He-style uniform initialisation (fan-in), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(3.0 / shape[1])
            p[name] = rng.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(theta, X, keep=False):
    """X: (B, 6) standardised inputs -> (B, 3) standardised outputs."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = gelu(z3)
    y = h3 @ p["W4"].T + p["b4"]
    if keep:
        return y, (X, z1, h1, z2, h2, z3, h3)
    return y


def loss(theta, X, Y):
    d = forward(theta, X) - Y
    return float(np.mean(d * d))


def backward(theta, X, Y):
    """Loss and its gradient w.r.t. the flat parameter vector."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2, z3, h3) = forward(theta, X, keep=True)
    B = X.shape[0]
    d = y - Y
    L = float(np.mean(d * d))
    dy = 2.0 * d / (B * NOUT)
    g = {}
    g["W4"] = dy.T @ h3
    g["b4"] = dy.sum(0)
    dz3 = (dy @ p["W4"]) * gelu_grad(z3)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return L, pack(g)


def bf16(a):
    """Round float64 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    r = ((u + rounding) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def quantised_forward(theta, X):
    """Forward with bfloat16 weights and activations, float64 accumulation."""
    p = unpack(theta)
    W = {k: bf16(v) if k.startswith("W") else v for k, v in p.items()}
    h = bf16(X)
    for i in (1, 2, 3):
        h = bf16(gelu(h @ W[f"W{i}"].T + W[f"b{i}"]))
    return h @ W["W4"].T + W["b4"]


def quantised_backward(theta, X, Y, rnd=bf16):
    """Loss and gradient of the network with bfloat16 operands (see the
    module docstring): the forward of ``quantised_forward``; dL/dy rounded;
    each layer's dZ = rnd((dZ_next W_next) * GELU'(z)) with the rounded
    weights; weight gradients dZ^T H and bias gradients sum(dZ) from the
    rounded dZ and activations.  ``rnd`` = identity gives ``backward``."""
    p = unpack(theta)
    B = X.shape[0]
    W = {k: rnd(v) for k, v in p.items() if k.startswith("W")}
    h = [rnd(X)]
    z = []
    for i in (1, 2, 3):
        z.append(h[-1] @ W[f"W{i}"].T + p[f"b{i}"])
        h.append(rnd(gelu(z[-1])))
    y = h[3] @ W["W4"].T + p["b4"]
    d = y - Y
    L = float(np.mean(d * d))
    dz = rnd(2.0 * d / (B * NOUT))
    g = {"W4": dz.T @ h[3], "b4": dz.sum(0)}
    for i in (3, 2, 1):
        dz = rnd((dz @ W[f"W{i + 1}"]) * gelu_grad(z[i - 1]))
        g[f"W{i}"] = dz.T @ h[i - 1]
        g[f"b{i}"] = dz.sum(0)
    return L, pack(g)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
