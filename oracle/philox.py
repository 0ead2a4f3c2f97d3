"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11).

Test infrastructure only.

The paper asks of its generator that every cell own a reproducible stream
independent of the process count, with small state and good statistics
(section on choosing a scalable parallel RNG).  A counter-based generator
meets this with no state at all: the block for a cell at a step is a pure
function of (counter, key).

Round function on the 4-word counter (c0, c1, c2, c3) with key (k0, k1):
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2      (64x64 -> 128-bit)
    c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
ten rounds, the key bumped by the Weyl constants (W0, W1) between rounds.

``block`` is the plain definition on Python integers; ``block_vec`` is the
same arithmetic on numpy uint64 arrays for many counters at once (the high
word of the product built from 32-bit halves).  Uniforms are u = (o >> 11) 2^-53.
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10


def block(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
    return (c0, c1, c2, c3)


def to_unit(o):
    """53-bit uniform in [0, 1) from one 64-bit output word."""
    return (int(o) >> 11) * (2.0 ** -53)


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    a = a.astype(np.uint64)
    b = np.uint64(b)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b   # wraps modulo 2^64
    return hi, lo


def block_vec(c0, c1, c2, c3, key):
    """Blocks for arrays of counter words (broadcast), returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        shape = c0.shape
        c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), shape).copy()
        c2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), shape).copy()
        c3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), shape).copy()
        c0 = c0.copy()
        k0, k1 = np.uint64(int(key[0]) & MASK64), np.uint64(int(key[1]) & MASK64)
        for r in range(ROUNDS):
            if r:
                k0 = np.uint64((int(k0) + W0) & MASK64)
                k1 = np.uint64((int(k1) + W1) & MASK64)
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def to_unit_vec(o):
    return (np.asarray(o, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
