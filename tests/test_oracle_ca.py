"""Pins of the oracle's cellular automaton (cellular module; CA numerical
treatment; conflict priority of Algorithm 2): SciPy's regularised incomplete
beta, a serial per-cell simulator run in every processing order on tiny
lattices, hand-worked cases and invariants."""
import itertools

import numpy as np
import pytest
from scipy.special import betainc

from oracle import ca, philox
from oracle.constants import (CANCER, CODE_KILL, CODE_NONE, CODE_NOSPACE, DEFAULT,
                              EMPTY, STREAM_KILL, STROMA)

P = DEFAULT


@pytest.mark.parametrize("b", [1, 2, 3, 5])
def test_kill_probability_is_incomplete_beta(b):
    x = np.linspace(0.0, 1.0, 101)
    np.testing.assert_allclose(ca.kill_probability(x, 1.0, b), betainc(1.0, b, x), atol=2e-16)
    # clipping of the normalised concentration
    assert ca.kill_probability(np.array([-0.3]), 1.0, b)[0] == 0.0
    assert ca.kill_probability(np.array([2.5]), 1.0, b)[0] == 1.0


# --------------------------------------------------------------------------
# serial simulator: one committed cell at a time, snapshot reads, conflicts
# settled by (phi desc, gid asc); written on coordinates, independent of the
# oracle's shifted-array machinery.

def serial_ca(L, w, K, G1, G2, phi, Pm, Vm, step, seed, p, order):
    nz, ny, nx = L.shape

    def gid(z, y, x):
        return x + nx * (y + ny * z)

    committed = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)
                 if L[z, y, x] == CANCER and phi[z, y, x] >= 1.0]
    cells = [committed[i] for i in order]
    fate = {}
    claims = {}
    for (z, y, x) in cells:
        g = gid(z, y, x)
        o = philox.block((g, step + 1, STREAM_KILL, 0), (seed, 0))
        u = [philox.to_unit(o[0]), philox.to_unit(o[1])]
        killed = False
        for i, G in enumerate((G1, G2)):
            xi = min(max(G[z, y, x] / p.G_ref[i], 0.0), 1.0)
            y_ = 1.0 - xi
            pw = y_
            for _ in range(p.b_int[i] - 1):
                pw = pw * y_
            if u[i] < 1.0 - pw:
                killed = True
        if killed:
            fate[(z, y, x)] = "kill"
            continue
        best, bestK = None, -np.inf
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dz, dy, dx) == (0, 0, 0):
                        continue
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
                        continue
                    if L[zz, yy, xx] != EMPTY or w[zz, yy, xx] != 0.0:
                        continue
                    if K[zz, yy, xx] > bestK:
                        best, bestK = (zz, yy, xx), K[zz, yy, xx]
        if best is None:
            fate[(z, y, x)] = "nospace"
            continue
        prio = (phi[z, y, x], -g)
        if best not in claims:
            claims[best] = ((z, y, x), prio)
            fate[(z, y, x)] = ("div", best)
        elif prio > claims[best][1]:
            fate[claims[best][0]] = "lost"
            claims[best] = ((z, y, x), prio)
            fate[(z, y, x)] = ("div", best)
        else:
            fate[(z, y, x)] = "lost"
    Ln, phin, Pn, Vn = L.copy(), phi.copy(), Pm.copy(), Vm.copy()
    for cell, f in fate.items():
        if f == "kill":
            Ln[cell] = EMPTY
            phin[cell] = Pn[cell] = Vn[cell] = 0.0
        elif f in ("nospace", "lost"):
            phin[cell] = 0.0
        else:
            t = f[1]
            phin[cell] = Pn[cell] = Vn[cell] = 0.0
            Ln[t] = CANCER
            phin[t] = Pn[t] = Vn[t] = 0.0
    return Ln, phin, Pn, Vn


def random_tiny_state(rng, shape, n_commit_max=6):
    L = rng.choice([EMPTY, CANCER, STROMA], size=shape, p=[0.45, 0.4, 0.15]).astype(np.uint8)
    w = np.where((L == EMPTY) & (rng.random(shape) < 0.2), rng.lognormal(0, 0.5, shape), 0.0)
    # coarse oxygen values to create ties
    K = rng.choice([5.0, 7.5, 7.5, 10.0], size=shape)
    G1 = rng.choice([0.0, 0.05, 0.3], size=shape)
    G2 = rng.choice([0.0, 0.02], size=shape)
    phi = rng.choice([0.2, 1.0, 1.3, 1.3], size=shape)
    cand = np.flatnonzero((L == CANCER).ravel() & (phi.ravel() >= 1.0))
    if cand.size > n_commit_max:
        drop = rng.choice(cand, size=cand.size - n_commit_max, replace=False)
        phi.ravel()[drop] = 0.5
    Pm = rng.random(shape)
    Vm = rng.random(shape)
    return L, w, K, G1, G2, phi, Pm, Vm


@pytest.mark.parametrize("trial", range(12))
def test_two_phase_equals_serial_in_every_order(trial):
    rng = np.random.default_rng(100 + trial)
    shape = [(2, 3, 3), (1, 3, 3), (2, 2, 3), (3, 3, 2)][trial % 4]
    L, w, K, G1, G2, phi, Pm, Vm = random_tiny_state(rng, shape)
    seed, step = 7 + trial, trial
    Ln, phin, Pn, Vn, _, _, _ = ca.ca_update(L, w, K, G1, G2, phi, Pm, Vm, step, seed, P)
    ncom = int(((L == CANCER) & (phi >= 1.0)).sum())
    for order in itertools.permutations(range(ncom)):
        s = serial_ca(L, w, K, G1, G2, phi, Pm, Vm, step, seed, P, order)
        for a, b in zip((Ln, phin, Pn, Vn), s):
            assert np.array_equal(a, b), order


def empty_state(shape):
    L = np.zeros(shape, dtype=np.uint8)
    w = np.zeros(shape)
    K = np.full(shape, 10.0)
    z = np.zeros(shape)
    return L, w, K, z.copy(), z.copy(), z.copy(), z.copy(), z.copy()


def test_uniform_oxygen_picks_lowest_gid_neighbour():
    L, w, K, G1, G2, phi, Pm, Vm = empty_state((3, 3, 3))
    L[1, 1, 1] = CANCER
    phi[1, 1, 1] = 1.0
    Ln, phin, *_ = ca.ca_update(L, w, K, G1, G2, phi, Pm, Vm, 0, 1, P)
    assert Ln[0, 0, 0] == CANCER and int(Ln.sum()) == 2
    assert phin[1, 1, 1] == 0.0


def test_highest_oxygen_neighbour_and_vessel_excluded():
    L, w, K, G1, G2, phi, Pm, Vm = empty_state((3, 3, 3))
    L[1, 1, 1] = CANCER
    phi[1, 1, 1] = 1.2
    K[2, 2, 2] = 19.0
    w[2, 2, 2] = 1.0            # best oxygen is a vessel: not allowed
    K[0, 2, 1] = 15.0
    Ln, *_ = ca.ca_update(L, w, K, G1, G2, phi, Pm, Vm, 0, 1, P)
    assert Ln[0, 2, 1] == CANCER and Ln[2, 2, 2] == EMPTY


def test_surrounded_cell_has_no_space():
    L, w, K, G1, G2, phi, Pm, Vm = empty_state((3, 3, 3))
    L[:] = STROMA
    L[1, 1, 1] = CANCER
    phi[1, 1, 1] = 1.5
    Pm[1, 1, 1], Vm[1, 1, 1] = 0.3, 0.4
    Ln, phin, Pn, Vn, ev, code, _ = ca.ca_update(L, w, K, G1, G2, phi, Pm, Vm, 0, 1, P)
    assert code[1, 1, 1] == CODE_NOSPACE and np.array_equal(Ln, L)
    assert phin[1, 1, 1] == 0.0 and Pn[1, 1, 1] == 0.3 and Vn[1, 1, 1] == 0.4


def test_conflict_higher_phi_wins_then_lower_gid():
    # 1-D row: parents at x=0 and x=2 both want x=1 (the only empty site)
    for phis, winner in [((1.2, 1.5), 2), ((1.5, 1.2), 0), ((1.3, 1.3), 0)]:
        L = np.array([[[CANCER, EMPTY, CANCER]]], dtype=np.uint8)
        w = np.zeros(L.shape)
        K = np.full(L.shape, 8.0)
        phi = np.array([[[phis[0], 0.0, phis[1]]]])
        z = np.zeros(L.shape)
        Ln, phin, Pn, Vn, ev, code, win = ca.ca_update(L, w, K, z, z, phi, z + 0.5, z + 0.5, 0, 1, P)
        assert Ln[0, 0, 1] == CANCER
        assert ev["divisions"] == 1 and ev["lost"] == 1
        loser = 2 - winner
        assert Pn[0, 0, winner] == 0.0 and Pn[0, 0, loser] == 0.5   # loser: only phi reset
        assert phin[0, 0, loser] == 0.0


def test_saturated_drug_always_kills_and_zero_drug_never():
    shape = (4, 6, 6)
    L = np.full(shape, CANCER, dtype=np.uint8)
    L[:, ::2, ::2] = EMPTY
    w = np.zeros(shape)
    K = np.full(shape, 10.0)
    phi = np.full(shape, 1.1)
    ones, zeros = np.ones(shape), np.zeros(shape)
    Ln, *_ , code, _ = ca.ca_update(L, w, K, ones, zeros, phi, zeros, zeros, 3, 9, P)
    assert np.all(code[L == CANCER] == CODE_KILL) and not np.any(Ln == CANCER)
    _, _, _, _, ev, code, _ = ca.ca_update(L, w, K, zeros, zeros, phi, zeros, zeros, 3, 9, P)
    assert ev["kills"] == 0


def test_kill_frequency_matches_probability():
    shape = (20, 50, 50)
    L = np.full(shape, CANCER, dtype=np.uint8)
    w, K = np.zeros(shape), np.full(shape, 10.0)
    G1 = np.full(shape, 0.3)
    G2 = np.full(shape, 0.1)
    phi = np.full(shape, 1.0)
    z = np.zeros(shape)
    code = ca.propose(L, w, K, G1, G2, phi, 5, 123, P)
    p_kill = 1.0 - (1.0 - 0.3) * (1.0 - 0.1)
    n = L.size
    frac = np.count_nonzero(code == CODE_KILL) / n
    assert abs(frac - p_kill) < 4.5 * np.sqrt(p_kill * (1 - p_kill) / n)


def test_invariants_on_a_random_lattice():
    rng = np.random.default_rng(11)
    shape = (6, 9, 8)
    L = rng.choice([0, 1, 2], size=shape, p=[0.4, 0.45, 0.15]).astype(np.uint8)
    w = np.where((L == 0) & (rng.random(shape) < 0.15), 1.0, 0.0)
    K = rng.random(shape) * 20
    G1 = rng.random(shape) * 0.2
    G2 = rng.random(shape) * 0.2
    phi = rng.random(shape) * 1.6
    Pm, Vm = rng.random(shape), rng.random(shape)
    Ln, phin, Pn, Vn, ev, code, win = ca.ca_update(L, w, K, G1, G2, phi, Pm, Vm, 2, 5, P)
    assert np.count_nonzero(Ln == STROMA) == np.count_nonzero(L == STROMA)
    assert np.all(Ln[w > 0] == EMPTY)
    dc = np.count_nonzero(Ln == CANCER) - np.count_nonzero(L == CANCER)
    assert dc == ev["divisions"] - ev["kills"]
    assert ev["divisions"] == np.count_nonzero(win != CODE_NONE)
    assert np.all(L[win != CODE_NONE] == EMPTY)
    # nothing committed -> nothing changes
    phi2 = np.minimum(phi, 0.99)
    Ln2, phin2, Pn2, Vn2, ev2, _, _ = ca.ca_update(L, w, K, G1, G2, phi2, Pm, Vm, 2, 5, P)
    assert np.array_equal(Ln2, L) and np.array_equal(phin2, phi2) and ev2["committed"] == 0
