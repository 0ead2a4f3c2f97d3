"""Pins of the oracle's theta-scheme substepping of Eqs. (oxygen) and (chemo)
inside one coupled step (Algorithm 1's PDE step, backward Euler or
Crank-Nicolson): the exact per-mode amplification factor of the scheme on
eigenvectors of the zero-flux Laplacian, convergence to the exact decay at
first (backward Euler) and second (Crank-Nicolson) order, the reaction-source
equilibrium as a fixed point, and the single backward-Euler substep as the
coupled step's system."""
import math

import numpy as np
import pytest

from oracle import lattice, model
from oracle.constants import DEFAULT as P

SHAPE = (4, 5, 6)   # (nz, ny, nx)
KMODE = (1, 2, 3)   # mode numbers along (z, y, x)


def mode(shape=SHAPE, kmode=KMODE):
    """Eigenvector of the zero-flux 7-point Laplacian (DCT-II basis) and its
    eigenvalue: Lap v = -lam v, lam = sum over axes of 2 - 2 cos(pi k / n)."""
    v = np.ones(shape)
    lam = 0.0
    for ax, (n, k) in enumerate(zip(shape, kmode)):
        x = (np.arange(n) + 0.5) * math.pi * k / n
        shape = [1, 1, 1]
        shape[ax] = n
        v = v * np.cos(x).reshape(shape)
        lam += 2.0 - 2.0 * math.cos(math.pi * k / n)
    return v, lam


def empty_state(G, K=None):
    z = np.zeros(G.shape)
    L = np.zeros(G.shape, dtype=np.uint8)
    return model.State(L, z.copy() if K is None else K, G.copy(), G.copy(), z.copy(), z.copy(), z.copy(), 0)


def test_mode_is_a_laplacian_eigenvector():
    v, lam = mode()
    np.testing.assert_allclose(lattice.laplacian_apply(v), -lam * v, atol=1e-13)


@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 1.0), (1, 0.5), (4, 0.5), (5, 0.7)])
def test_substeps_amplify_a_mode_by_the_theta_factor(m, theta):
    """No cells, no vessels, no drug in the plasma: each substep multiplies a
    Laplacian eigenvector by (1/tau - (1-theta) q) / (1/tau + theta q),
    q = psi + a lam (drugs) and a lam (oxygen, no uptake without cells)."""
    v, lam = mode()
    p = P.with_(pde_substeps=m, pde_theta=theta)
    tau = p.dt_min / m
    s = empty_state(v, K=2.0 * v)
    K, G1, G2 = model.solve_fields(s, np.zeros(SHAPE), model.Schedule(), p, method="lu")
    qg = p.psi_G + p.a_G * lam
    qk = p.a_K * lam
    ag = (1 / tau - (1 - theta) * qg) / (1 / tau + theta * qg)
    ak = (1 / tau - (1 - theta) * qk) / (1 / tau + theta * qk)
    np.testing.assert_allclose(G1, ag ** m * v, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(G2, ag ** m * v, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(K, 2.0 * ak ** m * v, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("theta,order", [(1.0, 1), (0.5, 2)])
def test_substeps_converge_to_the_exact_decay_at_the_scheme_order(theta, order):
    """Drug mode decay exp(-(psi + a lam) dt) of the slowest mode of a
    64-voxel line (q dt ~ 2): halving the substep halves the error of
    backward Euler and quarters that of Crank-Nicolson."""
    v, lam = mode((1, 1, 64), (0, 0, 1))
    q = P.psi_G + P.a_G * lam
    exact = math.exp(-q * P.dt_min)
    errs = []
    for m in (30, 60, 120):
        p = P.with_(pde_substeps=m, pde_theta=theta)
        _, G1, _ = model.solve_fields(empty_state(v), np.zeros(v.shape), model.Schedule(), p, method="lu")
        amp = float(np.sum(G1 * v) / np.sum(v * v))
        errs.append(abs(amp - exact))
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 == pytest.approx(2.0 ** order, rel=0.05), errs


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_reaction_source_equilibrium_is_a_fixed_point(theta):
    """Vessels everywhere with a constant plasma level g (no elimination):
    G* = kappa g / (psi + kappa) is stationary for any substep and theta."""
    p = P.with_(pde_substeps=3, pde_theta=theta, k_pk=(0.0, 0.0))
    w = np.ones(SHAPE)
    sched = model.Schedule(times=((0.0,), (0.0,)), amts=((1.5,), (0.5,)))
    g = (1.5 * p.G_ref[0], 0.5 * p.G_ref[1])
    G1s = p.kappa_G * g[0] / (p.psi_G + p.kappa_G)
    G2s = p.kappa_G * g[1] / (p.psi_G + p.kappa_G)
    s = empty_state(np.full(SHAPE, G1s), K=np.full(SHAPE, p.K0))
    s.G2[:] = G2s
    K, G1, G2 = model.solve_fields(s, w, sched, p, method="lu")
    np.testing.assert_allclose(G1, G1s, rtol=1e-13)
    np.testing.assert_allclose(G2, G2s, rtol=1e-13)
    np.testing.assert_allclose(K, p.K0, rtol=1e-13)   # no cells: K0 is the equilibrium


def test_one_backward_euler_substep_is_the_coupled_step_system():
    rng = np.random.default_rng(4)
    L = (rng.random(SHAPE) < 0.5).astype(np.uint8)
    w = np.where(L == 0, rng.random(SHAPE), 0.0)
    K = 1.0 + rng.random(SHAPE)
    G = rng.random(SHAPE)
    c1, b1 = model.o2_system(L, w, K, P)
    c2, b2 = model.o2_substep_system(L, w, K, P, P.dt_min, 1.0)
    np.testing.assert_allclose(c2, c1, rtol=1e-15)
    np.testing.assert_allclose(b2, b1, rtol=1e-15)
    c1, b1 = model.drug_system(w, G, 0.7, P)
    c2, b2 = model.drug_substep_system(w, G, 0.3, 0.7, P, P.dt_min, 1.0)
    np.testing.assert_allclose(c2, c1, rtol=1e-15)
    np.testing.assert_allclose(b2, b1, rtol=1e-15)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_plasma_levels_enter_at_the_substep_ends(theta):
    """A uniform field with vessels everywhere follows the scalar theta
    recursion of dG/dt = -R G + kappa g(t), R = psi + kappa, with the plasma
    level at each substep's start (weight 1 - theta) and end (theta): a bolus
    at 10 min enters in the first of three 10-min substeps only through its
    end level, then decays with the elimination rate."""
    m = 3
    p = P.with_(pde_substeps=m, pde_theta=theta)
    sched = model.Schedule(times=((10.0,), (20.0,)), amts=((2.0,), (1.0,)))
    w = np.ones(SHAPE)
    G0 = 0.25
    s = empty_state(np.full(SHAPE, G0), K=np.full(SHAPE, p.K0))
    _, G1, G2 = model.solve_fields(s, w, sched, p, method="lu")
    tau, R = p.dt_min / m, p.psi_G + p.kappa_G
    for i, G in ((0, G1), (1, G2)):
        tb, ab = sched.times[i][0], sched.amts[i][0]
        g = [ab * p.G_ref[i] * math.exp(-p.k_pk[i] * (t - tb)) if t >= tb else 0.0
             for t in (j * tau for j in range(m + 1))]
        x = G0
        for j in range(m):
            x = ((1 / tau - (1 - theta) * R) * x + p.kappa_G * (theta * g[j + 1] + (1 - theta) * g[j])) \
                / (1 / tau + theta * R)
        np.testing.assert_allclose(G, x, rtol=1e-12)


@pytest.fixture(scope="module")
def small_tissue():
    from paper_2105_00448_amd import synth
    return synth.make_tissue(10, 4, seed=5)


def nonlinear_o2_residual(L, w, K_old, K_new, p, tau, theta):
    """Residual of the implicit oxygen update with the uptake at the new value,
    written out term by term (theta scheme, explicit uptake at the old value)."""
    chi = (L != 0).astype(float)
    lhs = (K_new / tau + theta * p.r_k * w * K_new + theta * p.phi_K * chi * K_new / (p.K1 + K_new)
           - theta * p.a_K * lattice.laplacian_apply(K_new))
    rhs = (K_old / tau - (1 - theta) * (p.r_k * w * K_old + p.phi_K * chi * K_old / (p.K1 + K_old))
           + (1 - theta) * p.a_K * lattice.laplacian_apply(K_old) + p.r_k * w * p.K0)
    return (lhs - rhs) / np.abs(rhs).max()


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_newton_oxygen_solves_the_nonlinear_update(small_tissue, theta):
    """Newton steps on the uptake drive the residual of the nonlinear implicit
    update to rounding, converging quadratically; the linearised update (no
    Newton step) leaves a residual of the size of the linearisation gap."""
    t = small_tissue
    p0 = P.with_(pde_theta=theta)
    s = model.init_state(t.cell, t.w, 1, p0, method="lu")
    s.K *= 0.8   # away from the steady state, so the update moves K
    res = []
    for k in range(4):
        p = p0.with_(o2_newton=k)
        K, _, _ = model.solve_fields(s, t.w, model.Schedule(), p, method="lu")
        res.append(np.abs(nonlinear_o2_residual(t.cell, t.w, s.K, K, p, p.dt_min, theta)).max())
    assert res[0] > 1e-6                    # the linearisation gap is visible
    assert res[1] < 100 * res[0] ** 2       # quadratic convergence ...
    assert res[2] < 100 * res[1] ** 2
    assert res[3] < 1e-13                   # ... down to rounding


def test_uptake_continued_linearly_below_zero():
    """For K < 0 (reachable only through a theta < 1 substep's oscillation)
    the uptake is phi_K K/K1, the tangent at 0: the linearised coefficient is
    phi_K/K1, the oxygen diagonal stays >= 1/tau (an M-matrix), and the Newton
    terms join the K >= 0 ones continuously (C^1 at 0)."""
    shape = (2, 3, 4)
    L = np.ones(shape, dtype=np.uint8)
    w = np.zeros(shape)
    tau, theta = 15.0, 0.5
    Kneg = np.full(shape, -30.0)
    c, _ = model.o2_substep_system(L, w, Kneg, P, tau, theta)
    c0, _ = model.o2_substep_system(L, w, np.zeros(shape), P, tau, theta)
    assert np.array_equal(c, c0) and np.all(c >= 1.0 / tau)
    b_lin = np.ones(shape)
    for eps in (1e-7, 1e-9):
        cm, bm = model.o2_newton_system(L, w, np.full(shape, -eps), b_lin, P, tau, theta)
        cp, bp = model.o2_newton_system(L, w, np.full(shape, eps), b_lin, P, tau, theta)
        np.testing.assert_allclose(cm, cp, rtol=10 * eps)
        np.testing.assert_allclose(bm, bp, rtol=10 * eps)
    cn, bn = model.o2_newton_system(L, w, Kneg, b_lin, P, tau, theta)
    assert np.all(cn == c0) and np.all(bn == b_lin)      # linear uptake: no Newton correction


def test_crank_nicolson_after_vessel_changes_stays_well_posed():
    """Crank-Nicolson substeps right after vessel births and deaths (the
    stiff vessel source makes the scheme oscillate): every oxygen system keeps
    a positive diagonal and the fields stay finite."""
    from paper_2105_00448_amd import synth
    p = P.with_(vegf=1, pde_substeps=2, pde_theta=0.5, dv_min=60.0, V_high=5.0e-5, p_death=0.5,
                birth_per_V=0.4 / 5.0e-5)
    sched = model.Schedule(times=((0.0,), (0.0, 40.0)), amts=((1.0,), (1.0, 0.5)))
    tis = synth.make_tissue((2, 2, 130), 4, seed=138)
    s = model.init_state(tis.cell, tis.w, tis.seed, p)
    changes = 0
    for _ in range(4):
        c, _ = model.o2_substep_system(s.L, s.w, np.minimum(s.K, -1.0), p, 15.0, 0.5)
        assert c.min() > 0.0
        s, ev = model.step(s, None, sched, tis.seed, p)
        changes += ev["births"] + ev["deaths"]
        assert np.all(np.isfinite(s.K)) and np.all(np.isfinite(s.Vc))
    assert changes > 0
