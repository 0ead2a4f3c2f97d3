"""Pins of the oracle's intracellular ODEs (Eqs. odep53, odevegf, cellcycle)
and plasma kinetics (Eq. intrachemo3, fluorouracil model) against SciPy's
VODE (implicit Adams, the integrator the paper uses) and closed forms."""
import math

import numpy as np
import pytest
from scipy.integrate import ode as scipy_ode
from scipy.integrate import solve_ivp

from oracle import ode, pk
from oracle.constants import DEFAULT as PRM

KS = [0.0, 1e-9, 0.003, 0.01, 0.5, 6.9, 17.0, 20.0]


def vode_adams(rhs, y0, t1, max_step=1.0):
    r = scipy_ode(lambda t, y: rhs(t, y))
    r.set_integrator("vode", method="adams", rtol=1e-12, atol=1e-16, max_step=max_step,
                     nsteps=100000)
    r.set_initial_value(np.asarray(y0, dtype=float), 0.0)
    y = r.integrate(t1)
    assert r.successful()
    return y


def paper_rhs(K):
    """Right-hand sides of Eqs. (odep53), (odevegf), (cellcycle) as printed."""
    p = PRM

    def f(t, y):
        P, V, ph = y
        dP = p.k1 - p.k1p * K / (p.K_p53 + K) * P
        dV = p.k2 + p.k2pp * P * V / (p.J5 + V) - p.k2p * K / (p.K_V + K) * V
        dphi = K / (p.T_cycle * (p.K_phi + K))
        return [dP, dV, dphi]
    return f


@pytest.mark.parametrize("K", KS)
def test_step_matches_vode_adams(K):
    P0, V0, phi0 = 0.05, 0.3, 0.4
    ref = vode_adams(paper_rhs(K), [P0, V0, phi0], PRM.dt_min)
    Pn = ode.p53_exact(np.array([P0]), np.array([K]), PRM.dt_min, PRM)[0]
    Vn = ode.vegf_rk4(np.array([V0]), np.array([P0]), np.array([K]), PRM.dt_min,
                      PRM.ode_substeps, PRM)[0]
    phin = phi0 + ode.cycle_increment(np.array([K]), PRM.dt_min, PRM)[0]
    assert abs(Pn - ref[0]) <= 1e-10 * abs(ref[0])
    assert abs(Vn - ref[1]) <= 1e-9 * abs(ref[1])
    assert abs(phin - ref[2]) <= 1e-12 * abs(ref[2])


def test_vegf_linear_special_case_closed_form():
    """k2'' = 0 decouples V_c: V(t) = V_ss + (V0 - V_ss) exp(-mu t), V_ss = k2/mu."""
    p = PRM.with_(k2pp=0.0)
    K = np.array([0.02, 1.0, 15.0])
    V0 = np.array([0.0, 0.7, 0.05])
    mu = p.k2p * K / (p.K_V + K)
    exact = p.k2 / mu + (V0 - p.k2 / mu) * np.exp(-mu * p.dt_min)
    got = ode.vegf_rk4(V0, np.zeros(3), K, p.dt_min, p.ode_substeps, p)
    # RK4 truncation: about n (mu h)^5 / 120 relative, ~3e-11 here
    np.testing.assert_allclose(got, exact, rtol=1e-10)
    assert np.max(np.abs(got - exact) / exact) > 1e-14   # a real integrator, not the formula


@pytest.mark.parametrize("K", [0.05, 2.0, 6.9, 17.0, 20.0])
def test_steady_states_are_fixed_points_and_attractors(K):
    f = paper_rhs(K)
    Pss = ode.steady_p53(np.array([K]), PRM)[0]
    Vss = ode.steady_vegf(np.array([K]), np.array([Pss]), PRM)[0]
    d = f(0.0, [Pss, Vss, 0.0])
    assert abs(d[0]) < 1e-15 and abs(d[1]) < 1e-15
    # from far away the flow converges to the same point
    sol = solve_ivp(f, (0, 20000.0), [0.0, 0.0, 0.0], method="LSODA", rtol=1e-11, atol=1e-16)
    assert abs(sol.y[0, -1] - Pss) < 1e-8 * Pss
    assert abs(sol.y[1, -1] - Vss) < 1e-7 * Vss


def test_ode_step_touches_only_occupied_and_cycles_only_cancer():
    L = np.array([0, 1, 2, 1], dtype=np.uint8).reshape(1, 1, 4)
    K = np.array([10.0, 10.0, 10.0, 0.0]).reshape(1, 1, 4)
    P = np.full((1, 1, 4), 0.05)
    V = np.full((1, 1, 4), 0.2)
    phi = np.full((1, 1, 4), 0.5)
    Pn, Vn, phin = ode.ode_step(L, K, P, V, phi, PRM)
    assert Pn[0, 0, 0] == 0.05 and Vn[0, 0, 0] == 0.2 and phin[0, 0, 0] == 0.5
    assert phin[0, 0, 2] == 0.5            # stroma: no cycle
    assert phin[0, 0, 1] > 0.5 and phin[0, 0, 3] == 0.5   # K = 0: no progress
    assert Pn[0, 0, 3] == pytest.approx(0.05 + PRM.k1 * PRM.dt_min, rel=1e-14)


def test_plasma_matches_integrated_one_compartment_model():
    """Eq. (intrachemo3) integrated with resets at each bolus."""
    k, gref = PRM.k_pk[0], 1.0
    times, amts = (0.0, 1440.0, 2000.0), (1.0, 0.7, 1.3)
    probe = [0.0, 30.0, 700.0, 1439.0, 1440.0, 1900.0, 2000.0, 4000.0]
    # integrate piecewise
    def integrate_to(t):
        g, tc = 0.0, 0.0
        for tm, am in zip(times, amts):
            if tm > t:
                break
            if tm > tc:
                g = solve_ivp(lambda s, y: -k * y, (tc, tm), [g], rtol=1e-12, atol=1e-15).y[0, -1]
            g, tc = am * gref, tm
        if t > tc:
            g = solve_ivp(lambda s, y: -k * y, (tc, t), [g], rtol=1e-12, atol=1e-15).y[0, -1]
        return g
    for t in probe:
        ref = integrate_to(t)
        got = pk.plasma(t, times, amts, k, gref)
        assert abs(got - ref) <= 1e-9 * max(ref, 1e-300), (t, got, ref)
    assert pk.plasma(-1.0, times, amts, k, gref) == 0.0


def test_fluorouracil_linear_regime():
    """The Michaelis-Menten plasma model with G << k_m decays at v_max/k_m."""
    vmax, km = 1.75, 27.0
    g0 = 1e-3
    sol = solve_ivp(lambda t, y: -vmax / (km + y) * y, (0, 60.0), [g0], rtol=1e-12, atol=1e-18)
    lin = pk.plasma(60.0, (0.0,), (g0,), PRM.k_pk[1], 1.0)
    assert abs(sol.y[0, -1] - lin) < 1e-4 * lin


def test_fluorouracil_michaelis_menten_matches_integration():
    """The exact Michaelis-Menten plasma model (Lambert W closed form) against
    the integrated ODE with resets, in the nonlinear range G ~ k_m."""
    vmax, km = 1.75, 27.0
    times, amts = (0.0, 100.0, 2000.0), (60.0, 10.0, 27.0)
    def integrate_to(t):
        g, tc = 0.0, 0.0
        for tm, am in zip(times, amts):
            if tm > t:
                break
            if tm > tc:
                g = solve_ivp(lambda s, y: -vmax * y / (km + y), (tc, tm), [g], rtol=1e-12, atol=1e-18).y[0, -1]
            g, tc = am, tm
        if t > tc:
            g = solve_ivp(lambda s, y: -vmax * y / (km + y), (tc, t), [g], rtol=1e-12, atol=1e-18).y[0, -1]
        return g
    for t in (0.0, 5.0, 30.0, 99.0, 100.0, 130.0, 400.0, 2000.0, 2500.0):
        ref = integrate_to(t)
        got = pk.plasma_mm(t, times, amts, vmax, km, 1.0)
        assert abs(got - ref) <= 1e-9 * ref + 1e-15, (t, got, ref)
    assert pk.plasma_mm(-1.0, times, amts, vmax, km, 1.0) == 0.0


def test_fluorouracil_michaelis_menten_limits():
    """Small doses decay at the linear rate v_max/k_m; a dose far above k_m is
    first eliminated at the saturated rate v_max (zero order)."""
    vmax, km = 1.75, 27.0
    small = pk.plasma_mm(120.0, (0.0,), (1e-6,), vmax, km, 1.0)
    assert small == pytest.approx(1e-6 * math.exp(-vmax / km * 120.0), rel=1e-7)
    big = 1e6   # exp(G0/k_m) overflows: the large-argument branch
    g = pk.plasma_mm(10.0, (0.0,), (big,), vmax, km, 1.0)
    assert g == pytest.approx(big - vmax * 10.0, rel=1e-9)   # zero-order elimination
    # and the separated solution k_m ln(G/G0) + G - G0 = -v_max t holds to rounding
    assert abs(km * math.log(g / big) + g - big + vmax * 10.0) < 1e-8
