"""Parity of the HIP path's VEGF option with the oracle: the extracellular
VEGF field (Eq. vac_v without Avastin) solved in the same batch as oxygen and
the drugs, and the vessel birth-death update of the vascular module.

Fields: max-norm relative error <= 1e-10.  The vessel map, the cell map and
the event counts: bit-exact on shared inputs.
"""
import numpy as np
import pytest

from oracle import ca as oca
from oracle import model as om
from oracle import ode as oode
from oracle import vascular as ovas
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10
STATE = ("L", "K", "G1", "G2", "P", "Vc", "phi", "V", "w")


def relerr(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def vegf_params(op, **kw):
    base = dict(cg_rtol=1e-15, init_rtol=1e-15, cg_maxit=20000, init_maxit=400, vegf=1,
                V_high=op.V_high, p_death=op.p_death, birth_per_V=op.birth_per_V)
    base.update(kw)
    return hca.default_params(**base)


def push(sim, s):
    for name in STATE:
        sim.set_field(name, getattr(s, name))
    sim.set_step(s.step)


@pytest.fixture(scope="module")
def case32v():
    print("\n[case32v] 32^3, 8 Gaussians, seed 1, VEGF on", flush=True)
    tis = synth.make_tissue(32, 8, seed=1)
    sched = synth.DoseSchedule(times=((600.0,), (630.0,)), amts=((1.0,), (1.0,)))
    op = OP.with_(vegf=1, V_high=3.0e-5, p_death=0.5, birth_per_V=0.05 / 3.0e-5)
    s0 = om.init_state(tis.cell, tis.w, tis.seed, op)
    rng = np.random.default_rng(8)
    s0.V = 10.0 ** rng.uniform(-7.0, -4.0, size=s0.L.shape)   # spread over the window
    s0.step = 20
    return tis, sched, op, s0


def test_init_has_zero_vegf_and_the_input_vessels(case32v):
    tis, sched, op, _ = case32v
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))], vegf_params(op)) as sim:
        assert not sim.field("V").any()
        assert np.array_equal(sim.field("w"), tis.w)
        st = sim.stats()
        assert st["n_vessel"] == np.count_nonzero(tis.w) and st["total_births"] == 0


@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 0.5)], ids=["be1", "cn3"])
@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_vegf_field_matches_oracle(case32v, m, theta, precond):
    """V alone, then V batched with the other three fields: all four against
    the oracle."""
    print(f"\n[vegf] m {m} theta {theta} precond {precond}", flush=True)
    tis, sched, op, s0 = case32v
    opm = op.with_(pde_substeps=m, pde_theta=theta)
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    prm = vegf_params(opm, precond=precond, pde_substeps=m, pde_theta=theta)
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))], prm) as sim:
        push(sim, s0)
        sim.run_phases(hca.PH_VEGF)
        V = om.solve_vegf(s0, opm)
        assert relerr(sim.field("V"), V) <= FIELD_TOL
        assert sim.stats()["cg_iters_vegf"] > 0
        push(sim, s0)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS | hca.PH_VEGF)
        K, G1, G2 = om.solve_fields(s0, s0.w, osched, opm)
        for name, ref in (("K", K), ("G1", G1), ("G2", G2), ("V", V)):
            assert relerr(sim.field(name), ref) <= FIELD_TOL, name


@pytest.mark.parametrize("n", [23, 47, 5])
def test_vessel_update_bit_exact(case32v, n):
    """The CA and then the vessel update on a shared random state: cell map,
    cell state, vessel map and event counts bit-exact; no update off the
    update times (n = 5)."""
    tis, sched, op, s0 = case32v
    rng = np.random.default_rng(100 + n)
    shape = tis.cell.shape
    s = s0.copy()
    s.K = 5.0 + 15.0 * rng.random(shape)
    s.G1 = rng.random(shape) * 0.4
    s.G2 = rng.random(shape) * 0.2
    s.phi = np.where(s.L == 1, rng.choice([0.3, 0.99, 1.0, 1.2], size=shape), 0.0)
    s.step = n
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))], vegf_params(op)) as sim:
        push(sim, s)
        sim.run_phases(hca.PH_CA | hca.PH_STATS)
        Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, s.w, s.K, s.G1, s.G2, s.phi, s.P, s.Vc, n,
                                                   tis.seed, op)
        wn, nb, nd = ovas.vessel_update(Ln, s.w, s.V, n, tis.seed, op)
        assert np.array_equal(sim.field("L"), Ln)
        assert np.array_equal(sim.field("phi"), phin)
        assert np.array_equal(sim.field("P"), Pn) and np.array_equal(sim.field("Vc"), Vn)
        assert np.array_equal(sim.field("w"), wn)
        st = sim.stats()
        assert (st["vessel_births"], st["vessel_deaths"]) == (nb, nd)
        assert st["n_vessel"] == np.count_nonzero(wn)
        if n == 5:
            assert nb == nd == 0
        else:
            assert nb > 0 and nd > 0


@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_vegf_trajectory_resynchronised(case32v, precond):
    """Steps 20..27 with the VEGF option (vessel update at the end of step
    23 -> 24): each step's four solves and ODE at the field tolerance, the CA
    and the vessel update bit-exact; the GPU restarts every step from the
    oracle's state."""
    tis, sched, op, s0 = case32v
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = s0
    births = deaths = 0
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))],
                        vegf_params(op, precond=precond)) as sim:
        for n in range(8):
            push(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS | hca.PH_VEGF)
            K, G1, G2 = om.solve_fields(s, s.w, osched, op)
            V = om.solve_vegf(s, op)
            for name, ref in (("K", K), ("G1", G1), ("G2", G2), ("V", V)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
                sim.set_field(name, ref)
            sim.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, op)
            Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, s.w, K, G1, G2, phi, P, Vc, s.step,
                                                       tis.seed, op)
            wn, nb, nd = ovas.vessel_update(Ln, s.w, V, s.step, tis.seed, op)
            assert np.array_equal(sim.field("L"), Ln), n
            assert np.array_equal(sim.field("phi"), phin), n
            assert relerr(sim.field("P"), Pn) <= FIELD_TOL
            assert relerr(sim.field("Vc"), Vn) <= FIELD_TOL
            assert np.array_equal(sim.field("w"), wn), n
            st = sim.stats()
            assert (st["vessel_births"], st["vessel_deaths"]) == (nb, nd), n
            births += nb
            deaths += nd
            s = om.State(Ln, K, G1, G2, Pn, Vn, phin, s.step + 1, V, wn)
    assert births > 0 and deaths > 0


def test_vegf_full_steps_match_oracle_steps(case32v):
    """hca_step (all phases) over the vessel update against the oracle's
    step, restarting from the oracle's state each step."""
    tis, sched, op, s0 = case32v
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = s0
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))], vegf_params(op)) as sim:
        for n in range(4):
            push(sim, s)
            sim.step(1)
            s, ev = om.step(s, None, osched, tis.seed, op)
            assert np.array_equal(sim.field("w"), s.w), n
            assert relerr(sim.field("V"), s.V) <= FIELD_TOL, n
            st = sim.stats()
            assert st["step"] == s.step and st["vessel_births"] == ev["births"]


def test_vessel_map_setter_validates(case32v):
    tis, sched, op, _ = case32v
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))], vegf_params(op)) as sim:
        bad = tis.w.copy()
        bad.ravel()[np.flatnonzero(tis.cell)[0]] = 1.0      # a vessel on a cell
        with pytest.raises(RuntimeError):
            sim.set_field("w", bad)
        neg = tis.w.copy()
        neg.ravel()[np.flatnonzero(tis.cell == 0)[0]] = -1.0
        with pytest.raises(RuntimeError):
            sim.set_field("w", neg)
        assert np.array_equal(sim.field("w"), tis.w)        # unchanged
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))],
                        vegf_params(op, vegf=0)) as sim:
        with pytest.raises(RuntimeError):
            sim.field("V")
