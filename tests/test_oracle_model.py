"""Pins of the oracle's Algorithm 1 (initialisation and coupled step):
reduction to a plain linear solve, fixed-point residuals, maximum principles
and cell-count bookkeeping."""
import numpy as np
import pytest

from oracle import lattice, model, ode
from oracle.constants import CANCER, DEFAULT as P, STROMA
from paper_2105_00448_amd import synth


@pytest.fixture(scope="module")
def tissue():
    return synth.make_tissue(12, 4, seed=3)


def test_steady_oxygen_without_cells_is_one_linear_solve(tissue):
    L0 = np.zeros_like(tissue.cell)
    K, its = model.steady_oxygen(L0, tissue.w, P)
    direct = lattice.solve(P.r_k * tissue.w, P.a_K, P.r_k * tissue.w * P.K0)
    np.testing.assert_allclose(K, direct, rtol=1e-13)
    # no uptake and a source everywhere the vessels are: K = K0 everywhere
    np.testing.assert_allclose(K, P.K0, rtol=1e-12)
    assert its <= 3


def test_steady_oxygen_is_a_fixed_point(tissue):
    K, _ = model.steady_oxygen(tissue.cell, tissue.w, P)
    chi = (tissue.cell != 0).astype(float)
    # nonlinear residual of Eq. (oxygen) with s_K = 0, written independently
    res = (P.a_K * lattice.laplacian_apply(K) - P.phi_K * K / (P.K1 + K) * chi
           + P.r_k * tissue.w * (P.K0 - K))
    scale = P.r_k * (tissue.w * P.K0).max()
    assert np.abs(res).max() < 1e-12 * scale
    assert K.min() > 0.0 and K.max() <= P.K0 * (1 + 1e-14)


def test_init_state(tissue):
    s = model.init_state(tissue.cell, tissue.w, seed=5, p=P)
    occ = tissue.cell != 0
    can = tissue.cell == CANCER
    assert np.all(s.P[~occ] == 0) and np.all(s.Vc[~occ] == 0) and np.all(s.phi[~can] == 0)
    assert s.phi[can].min() >= 0.0 and s.phi[can].max() < 1.0
    # P, V_c are the ODE steady states: the right-hand sides vanish
    K = s.K[occ]
    dP = P.k1 - P.k1p * K / (P.K_p53 + K) * s.P[occ]
    dV = P.k2 + P.k2pp * s.P[occ] * s.Vc[occ] / (P.J5 + s.Vc[occ]) - P.k2p * K / (P.K_V + K) * s.Vc[occ]
    assert np.abs(dP).max() < 1e-16 and np.abs(dV).max() < 1e-16
    assert np.all(s.G1 == 0) and np.all(s.G2 == 0)


def test_steps_keep_invariants(tissue):
    sched = model.Schedule(times=((0.0,), (0.0,)), amts=((1.0,), (0.8,)))
    s = model.init_state(tissue.cell, tissue.w, seed=5, p=P)
    n_stroma = np.count_nonzero(s.L == STROMA)
    gmax = 0.0
    for n in range(6):
        nc = np.count_nonzero(s.L == CANCER)
        Lold = s.L
        s, ev = model.step(s, tissue.w, sched, 5, P)
        assert np.count_nonzero(s.L == STROMA) == n_stroma
        assert np.count_nonzero(s.L == CANCER) - nc == ev["divisions"] - ev["kills"]
        assert np.all(s.L[tissue.w > 0] == 0)
        # maximum principles of the M-matrix systems
        assert s.K.min() > 0 and s.K.max() <= P.K0 * (1 + 1e-13)
        g0 = model.plasma_pair((n + 1) * P.dt_min, sched, P)
        gmax = max(gmax, g0[0])
        assert s.G1.min() >= 0 and s.G1.max() <= gmax * (1 + 1e-13)
    assert s.step == 6


def test_no_drug_no_commit_keeps_the_cell_map(tissue):
    s = model.init_state(tissue.cell, tissue.w, seed=5, p=P)
    s.phi[:] = 0.0
    s2, ev = model.step(s, tissue.w, model.Schedule(), 5, P)
    assert ev["committed"] == 0 and np.array_equal(s2.L, s.L)
    assert np.all(s2.G1 == 0)


def test_lu_and_cg_paths_agree(tissue):
    s = model.init_state(tissue.cell, tissue.w, seed=5, p=P)
    sched = model.Schedule(times=((0.0,), (0.0,)), amts=((1.0,), (1.0,)))
    a = model.solve_fields(s, tissue.w, sched, P, method="lu")
    b = model.solve_fields(s, tissue.w, sched, P, method="cg")
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-11 * np.abs(x).max()
