"""Pins of the oracle's Philox4x64-10 (Salmon et al., SC'11) against the
published known-answer vector and NumPy's independent implementation."""
import os

import numpy as np
import pytest

from oracle import philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def read_kat():
    vals = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        tag, *words = line.split()
        vals[tag] = [int(w, 16) for w in words]
    return vals


def numpy_block(ctr, key):
    """NumPy's Philox emits the block of (counter + 1) first, so start one below."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    k = sum(int(w) << (64 * i) for i, w in enumerate(key))
    g = np.random.Philox(counter=(c - 1) % (1 << 256), key=k)
    return tuple(int(x) for x in g.random_raw(4))


def test_known_answer_vector():
    kat = read_kat()
    assert philox.block(kat["ctr"], kat["key"]) == tuple(kat["out"])


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((12345, 7, 1, 0), (1, 0)),
    ((2 ** 64 - 1, 2 ** 64 - 1, 5, 9), (2 ** 63 + 11, 77)),
    ((32767, 20, 1, 0), (1000, 0)),
    ((56_623_103, 200, 0, 0), (2 ** 40, 0)),
])
def test_matches_numpy(ctr, key):
    assert philox.block(ctr, key) == numpy_block(ctr, key)


def test_vectorised_equals_scalar():
    rng = np.random.default_rng(0)
    gids = rng.integers(0, 2 ** 63, size=64, dtype=np.int64).astype(np.uint64)
    for step, stream, key in [(1, 1, (1, 0)), (99, 0, (2 ** 64 - 3, 0))]:
        v = philox.block_vec(gids, step, stream, 0, key)
        for i, g in enumerate(gids):
            s = philox.block((int(g), step, stream, 0), key)
            assert tuple(int(v[j][i]) for j in range(4)) == s


def test_uniforms_in_unit_interval_and_uniform():
    gids = np.arange(200000, dtype=np.uint64)
    o0, o1, _, _ = philox.block_vec(gids, 3, 1, 0, (42, 0))
    u = philox.to_unit_vec(o0)
    assert u.min() >= 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    expected = len(u) / 20
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert chi2 < 45.0          # 19 dof, p ~ 1e-3
    assert philox.to_unit(int(o1[5])) == philox.to_unit_vec(o1[5:6])[0]
