"""Pins of the oracle's third drug (epirubicin): the three-compartment plasma
kinetics against an independent integration of the model with resets, its
one-compartment limit and the sum of exponentials from the eigenvectors of
the rate matrix; the tissue field's vessel-source equilibrium; the third
kill trial (certain kill at G3 = G_ref3, no effect at G3 = 0, frequency
within a binomial bound)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ca, model, pk
from oracle.constants import CANCER
from oracle.constants import DEFAULT as P

P3 = P.with_(drug3=1)
TIMES = (0.0, 180.0, 2000.0)
AMTS = (1.0, 0.6, 0.8)


def rates(p):
    k10, k12, k13 = p.epi_cl / p.epi_w1, p.epi_q2 / p.epi_w1, p.epi_q3 / p.epi_w1
    k21, k31 = p.epi_q2 / p.epi_w2, p.epi_q3 / p.epi_w3
    return k10, k12, k13, k21, k31


def integrate(t, p, times=TIMES, amts=AMTS):
    """The three ODEs as written (plasma outflow on G0) by an implicit
    integrator, state carried across the boluses, G0 reset at each."""
    k10, k12, k13, k21, k31 = rates(p)

    def rhs(_, y):
        g0, g1, g2 = y
        return [-(k10 + k12 + k13) * g0 + k21 * g1 + k31 * g2, k12 * g0 - k21 * g1, k13 * g0 - k31 * g2]

    y, tc = np.zeros(3), None
    for tm, am in zip(times, amts):
        if tm > t:
            break
        if tc is not None and tm > tc:
            y = solve_ivp(rhs, (tc, tm), y, method="Radau", rtol=1e-12, atol=1e-16).y[:, -1]
        y = y.copy()
        y[0] = am * p.G_ref3
        tc = tm
    if tc is None:
        return 0.0
    if t > tc:
        y = solve_ivp(rhs, (tc, t), y, method="Radau", rtol=1e-12, atol=1e-16).y[:, -1]
    return y[0]


def test_plasma_matches_integration_with_resets():
    for t in (0.0, 1.0, 30.0, 179.0, 180.0, 181.0, 600.0, 1999.0, 2000.0, 2600.0, 10000.0):
        ref = integrate(t, P3)
        got = pk.plasma_epi(t, TIMES, AMTS, P3)
        assert abs(got - ref) <= 1e-9 * max(ref, 1e-6), (t, got, ref)
    assert pk.plasma_epi(-1.0, TIMES, AMTS, P3) == 0.0
    assert pk.plasma_epi(180.0, TIMES, AMTS, P3) == pytest.approx(0.6, rel=1e-15)   # reset level


def test_peripheral_content_survives_a_bolus():
    """After the second bolus the level exceeds a fresh single dose of the
    same size: the peripheral compartments return drug to the plasma."""
    fresh = pk.plasma_epi(600.0 - 180.0, (0.0,), (0.6,), P3)
    assert pk.plasma_epi(600.0, TIMES, AMTS, P3) > fresh * (1.0 + 1e-3)


def test_one_compartment_limit():
    p = P3.with_(epi_q2=0.0, epi_q3=0.0)
    k = p.epi_cl / p.epi_w1
    for t in (0.0, 10.0, 100.0, 179.0):
        assert pk.plasma_epi(t, (0.0,), (0.7,), p) == pytest.approx(0.7 * math.exp(-k * t), rel=1e-12)


def test_sum_of_exponentials():
    """A single bolus: G0(t) = sum_i c_i exp(lambda_i t) with lambda_i, c_i
    from the eigen-decomposition of the rate matrix (the closed form)."""
    M = pk.epi_rate_matrix(P3)
    lam, S = np.linalg.eig(M)
    assert np.all(lam.real < 0) and np.allclose(lam.imag, 0)
    c = S[0, :] * np.linalg.solve(S, np.array([1.0, 0.0, 0.0]))
    for t in (5.0, 60.0, 500.0, 5000.0):
        ref = float(np.real(np.sum(c * np.exp(lam * t))))
        assert pk.plasma_epi(t, (0.0,), (1.0,), P3) == pytest.approx(ref, rel=1e-10)


def test_third_drug_field_source_equilibrium():
    """Every voxel a vessel of weight w0, no cells, a plasma level held
    constant (no elimination or exchange): G3 = kappa w0 g/(psi + kappa w0)
    is the fixed point of every scheme."""
    shape = (3, 4, 5)
    p = P3.with_(epi_cl=0.0, epi_q2=0.0, epi_q3=0.0)
    w0, g = 0.8, 0.9
    geq = p.kappa_G * w0 * g / (p.psi_G + p.kappa_G * w0)
    L = np.zeros(shape, dtype=np.uint8)
    z = np.zeros(shape)
    sched = model.Schedule(times=((), (), (0.0,)), amts=((), (), (g,)))
    for m, theta in ((1, 1.0), (3, 0.5)):
        pm = p.with_(pde_substeps=m, pde_theta=theta)
        s = model.State(L, z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), 2,
                        G3=np.full(shape, geq))
        G3 = model.solve_drug3(s, np.full(shape, w0), sched, pm, method="lu")
        np.testing.assert_allclose(G3, geq, rtol=1e-12)


def committed_state(shape, rng):
    L = np.full(shape, CANCER, dtype=np.uint8)
    phi = np.full(shape, 1.5)
    z = np.zeros(shape)
    K = rng.random(shape)
    return L, phi, z, K


def test_third_kill_trial():
    shape = (8, 16, 16)
    rng = np.random.default_rng(3)
    L, phi, z, K = committed_state(shape, rng)
    w = np.zeros(shape)
    # certain kill at G3 = G_ref3
    code = ca.propose(L, w, K, z, z, phi, 4, 9, P3, G3=np.full(shape, P3.G_ref3))
    assert np.all(code == ca.CODE_KILL)
    # no third drug in the tissue: identical to the two-drug automaton
    G1 = rng.random(shape) * 0.3
    a = ca.propose(L, w, K, G1, z, phi, 4, 9, P3, G3=z)
    b = ca.propose(L, w, K, G1, z, phi, 4, 9, P)
    assert np.array_equal(a, b)
    # frequency: p3 = 1 - (1 - 0.3) = 0.3 with G1 = G2 = 0
    code = ca.propose(L, w, K, z, z, phi, 4, 9, P3, G3=np.full(shape, 0.3))
    n = L.size
    kills = np.count_nonzero(code == ca.CODE_KILL)
    assert abs(kills - 0.3 * n) < 5 * math.sqrt(n * 0.3 * 0.7)
