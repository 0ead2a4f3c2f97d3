"""Helpers shared by the surrogate's GPU tests: the oracle's quantised
forward with a per-output bound on the library's evaluation of it, and a
network descriptor of host parameters."""
import numpy as np

from oracle import mlp as omlp
from paper_2105_00448_amd import hca


def quantised_forward_bound(theta, Xs):
    """The oracle's quantised forward y of the standardised rows Xs and, per
    row and output, a bound E on |y_gpu - y| for the library's evaluation
    (FP32 accumulation, GELU from its table).  Layer by layer: the kernel's
    pre-activation z differs from the oracle's by at most Ez = sum |W| Eh
    (the previous layer's activation differences) + 65 2^-24 sum |W h| +
    |b| (FP32 accumulation of <= 64 products and the bias); the value it
    rounds, GELU(z), by at most ev = 1.01 |GELU'(z)| Ez + 8e-6 |z| (the
    table's Phi is within 7.5e-6) + 2^-23 |GELU(z)|.  Rounding to bfloat16
    is monotone, so the kernel's activation equals the oracle's unless
    [GELU(z) - ev, GELU(z) + ev] holds a rounding boundary; then it differs by
    at most the larger of the end values' rounding shifts, Eh.  The inputs
    and weights are rounded identically on both sides (Eh = 0 there)."""
    q = omlp.bf16
    p = omlp.unpack(theta)
    W = {k: q(v) for k, v in p.items() if k.startswith("W")}
    gam = 65 * 2.0 ** -24
    h = q(Xs)
    Eh = np.zeros_like(h)
    for i in (1, 2, 3):
        Wi, bi = W[f"W{i}"], p[f"b{i}"]
        z = h @ Wi.T + bi
        Ez = Eh @ np.abs(Wi).T + gam * (np.abs(h) @ np.abs(Wi).T + np.abs(bi))
        v = omlp.gelu(z)
        ev = 1.01 * np.abs(omlp.gelu_grad(z)) * Ez + 8e-6 * np.abs(z) + 2.0 ** -23 * np.abs(v)
        hq = q(v)
        Eh = np.maximum(np.abs(q(v + ev) - hq), np.abs(q(v - ev) - hq))
        h = hq
    W4, b4 = W["W4"], p["b4"]
    y = h @ W4.T + b4
    Ey = Eh @ np.abs(W4).T + gam * (np.abs(h) @ np.abs(W4).T + np.abs(b4))
    return y, Ey


def host_net(theta, stats):
    """An Mlp descriptor of FP32 host parameters (kept alive by the caller
    through the returned array) and the given statistics, box check off."""
    net = hca.Mlp()
    th32 = np.ascontiguousarray(theta, dtype=np.float32)
    net.theta = th32.ctypes.data
    net.theta_is_device = 0
    for k, v in stats.items():
        arr = getattr(net, k)
        for i, x in enumerate(v):
            arr[i] = float(x)
    net.box_check = 0
    return net, th32
