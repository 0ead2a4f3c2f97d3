"""Pins of the oracle's extracellular VEGF, Eq. (vac_v) without Avastin, and of
the vessel birth-death update of the vascular module, Eq. (vascular_module).

VEGF: the exact per-mode amplification factor of the theta scheme on
eigenvectors of the zero-flux Laplacian (decay and diffusion), the global mass
balance of the secretion (the zero-flux Laplacian sums to zero), and the
uniform secretion-decay equilibrium a V_c / psi_V as a fixed point.
Vessels: a second, voxel-by-voxel transcription on coordinates with the
scalar Philox; the extreme probabilities 0 and 1 and the window's closed ends;
event frequencies within binomial bounds; no update between update times;
births only on empty non-vessel voxels, deaths only outside the window; and
V's one-way coupling (the other fields and the CA do not see it)."""
import math

import numpy as np
import pytest

from oracle import model, vascular
from oracle.constants import DEFAULT as P
from oracle.constants import EMPTY, CANCER, STROMA
from paper_2105_00448_amd import synth

SHAPE = (4, 5, 6)   # (nz, ny, nx)


def mode(shape=SHAPE, kmode=(1, 2, 3)):
    v = np.ones(shape)
    lam = 0.0
    for ax, (n, k) in enumerate(zip(shape, kmode)):
        x = (np.arange(n) + 0.5) * math.pi * k / n
        sh = [1, 1, 1]
        sh[ax] = n
        v = v * np.cos(x).reshape(sh)
        lam += 2.0 - 2.0 * math.cos(math.pi * k / n)
    return v, lam


def vstate(L, V, Vc):
    z = np.zeros(L.shape)
    return model.State(L, z.copy(), z.copy(), z.copy(), z.copy(), Vc, z.copy(), 0, V, None)


@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 1.0), (1, 0.5), (4, 0.5), (2, 0.7)])
def test_vegf_mode_amplification(m, theta):
    """No cells: each substep multiplies a Laplacian eigenvector (eigenvalue
    -lam) by (1/tau - (1-theta) q)/(1/tau + theta q), q = psi_V + a_V lam."""
    v, lam = mode()
    p = P.with_(vegf=1, pde_substeps=m, pde_theta=theta)
    tau = p.dt_min / m
    L = np.zeros(SHAPE, dtype=np.uint8)
    V = model.solve_vegf(vstate(L, 3e-5 * v, np.zeros(SHAPE)), p, method="lu")
    q = p.psi_V + p.a_V * lam
    amp = (1 / tau - (1 - theta) * q) / (1 / tau + theta * q)
    np.testing.assert_allclose(V, amp ** m * 3e-5 * v, rtol=1e-11, atol=1e-20)


@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 0.5), (2, 0.7)])
def test_vegf_mass_balance(m, theta):
    """Summed over the lattice the diffusion drops out, so the total M obeys
    M' = (M (1/tau - (1-theta) psi_V) + a sum(V_c chi)) / (1/tau + theta psi_V)
    per substep, for any cell map and V_c."""
    rng = np.random.default_rng(3)
    L = rng.choice([EMPTY, CANCER, STROMA], size=SHAPE).astype(np.uint8)
    Vc = np.where(L != 0, rng.random(SHAPE), 0.0)
    V0 = 1e-4 * rng.random(SHAPE)
    p = P.with_(vegf=1, pde_substeps=m, pde_theta=theta)
    tau = p.dt_min / m
    V = model.solve_vegf(vstate(L, V0, Vc), p, method="lu")
    M = V0.sum()
    src = p.sec_V * Vc[L != 0].sum()
    for _ in range(m):
        M = (M * (1 / tau - (1 - theta) * p.psi_V) + src) / (1 / tau + theta * p.psi_V)
    assert abs(V.sum() - M) <= 1e-12 * M


def test_vegf_uniform_equilibrium_is_a_fixed_point():
    """A fully occupied lattice with uniform V_c: V = a V_c / psi_V balances
    secretion and decay and has no gradient, so every scheme keeps it."""
    L = np.full(SHAPE, CANCER, dtype=np.uint8)
    Vc = np.full(SHAPE, 0.2)
    for m, theta in ((1, 1.0), (3, 0.5)):
        p = P.with_(vegf=1, pde_substeps=m, pde_theta=theta)
        Veq = np.full(SHAPE, p.sec_V * 0.2 / p.psi_V)
        V = model.solve_vegf(vstate(L, Veq, Vc), p, method="lu")
        np.testing.assert_allclose(V, Veq, rtol=1e-12)


def random_vascular_state(rng, shape, p):
    L = rng.choice([EMPTY, EMPTY, CANCER, STROMA], size=shape).astype(np.uint8)
    w = np.where((L == EMPTY) & (rng.random(shape) < 0.4), 0.5 + rng.random(shape), 0.0)
    # V spread over and around the window, with both closed ends hit exactly
    V = 10.0 ** rng.uniform(-7.0, -3.0, size=shape)
    V.ravel()[::7] = p.V_low
    V.ravel()[3::11] = p.V_high
    return L, w, V


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vessel_update_matches_voxel_loop(seed):
    rng = np.random.default_rng(seed)
    p = P.with_(vegf=1, p_death=0.4, birth_per_V=0.5 / P.V_high)
    L, w, V = random_vascular_state(rng, (4, 6, 8), p)
    n = 24 * (seed + 1) - 1
    a = vascular.vessel_update(L, w, V, n, 11 + seed, p)
    b = vascular.vessel_update_serial(L, w, V, n, 11 + seed, p)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    assert a[1] > 0 and a[2] > 0


def test_vessel_update_extremes_and_window_ends():
    rng = np.random.default_rng(5)
    shape = (4, 6, 7)
    L, w, V = random_vascular_state(rng, shape, P)
    inside = (V >= P.V_low) & (V <= P.V_high)
    free = (w == 0) & (L == EMPTY)
    # probability 1: every vessel outside the window dies; birth_per_V V = 1 at
    # V = V_high, so every free voxel at exactly V_high is born
    p = P.with_(vegf=1, p_death=1.0, birth_per_V=1.0 / P.V_high)
    wn, nb, nd = vascular.vessel_update(L, w, V, 23, 9, p)
    assert np.all(wn[(w > 0) & ~inside] == 0.0) and nd == np.count_nonzero((w > 0) & ~inside)
    assert np.all(wn[(w > 0) & inside] == w[(w > 0) & inside])     # the window is closed at both ends
    assert np.all(wn[free & (V == P.V_high)] == p.w_new)
    assert np.all(wn[free & ~inside] == 0.0)
    assert np.all(wn[L != EMPTY] == 0.0)                            # never on a cell
    # probability 0: nothing happens
    p0 = P.with_(vegf=1, p_death=0.0, birth_per_V=0.0)
    wn, nb, nd = vascular.vessel_update(L, w, V, 23, 9, p0)
    assert np.array_equal(wn, w) and nb == nd == 0


def test_vessel_update_only_at_update_times():
    rng = np.random.default_rng(6)
    p = P.with_(vegf=1, p_death=1.0, birth_per_V=1.0 / P.V_high)
    L, w, V = random_vascular_state(rng, (3, 4, 5), p)
    assert p.dv_steps == 24
    for n in (0, 1, 22, 24, 46):
        wn, nb, nd = vascular.vessel_update(L, w, V, n, 1, p)
        assert np.array_equal(wn, w) and nb == nd == 0
    for n in (23, 47):
        wn, nb, nd = vascular.vessel_update(L, w, V, n, 1, p)
        assert nd > 0


def test_vessel_event_frequencies():
    """Deaths at rate p_death among vessels outside the window, births at
    rate birth_per_V V among free voxels inside it (5-sigma binomial bounds)."""
    shape = (16, 64, 64)
    rng = np.random.default_rng(7)
    p = P.with_(vegf=1, p_death=0.3, birth_per_V=0.5 / P.V_high)
    L = np.zeros(shape, dtype=np.uint8)
    w = np.where(rng.random(shape) < 0.5, 1.0, 0.0)
    V = np.where(w > 0, 2.0 * p.V_high, rng.uniform(p.V_low, p.V_high, size=shape))
    wn, nb, nd = vascular.vessel_update(L, w, V, 23, 123, p)
    nv = np.count_nonzero(w)
    assert abs(nd - p.p_death * nv) < 5 * math.sqrt(nv * p.p_death * (1 - p.p_death))
    pb = p.birth_per_V * V[w == 0]
    mean, var = pb.sum(), (pb * (1 - pb)).sum()
    assert abs(nb - mean) < 5 * math.sqrt(var)


def test_vegf_is_one_way_coupled():
    """With the VEGF option the step's K, G1, G2, P, V_c, phi and cell map are
    those of the plain step (V enters only the vessel update), and between
    update times the vessel map is unchanged."""
    tis = synth.make_tissue(12, 2, seed=4)
    pv = P.with_(vegf=1)
    s0 = model.init_state(tis.cell, tis.w, tis.seed, P)
    s1 = model.init_state(tis.cell, tis.w, tis.seed, pv)
    assert s1.V is not None and not s1.V.any() and np.array_equal(s1.w, tis.w)
    sched = model.Schedule(times=((0.0,), (0.0,)), amts=((1.0,), (1.0,)))
    for _ in range(2):
        s0, e0 = model.step(s0, tis.w, sched, tis.seed, P)
        s1, e1 = model.step(s1, tis.w, sched, tis.seed, pv)
        for name in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
            assert np.array_equal(getattr(s0, name), getattr(s1, name)), name
        assert np.array_equal(s1.w, tis.w) and e1["births"] == e1["deaths"] == 0
        assert s1.V.min() > 0.0
