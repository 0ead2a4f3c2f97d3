"""Parity of the HIP path's third drug (epirubicin) with the oracle: its
three-compartment plasma level seen through the tissue field G3, solved in
the same batch as the other fields; the third kill trial of the automaton;
and full steps with the third drug and the VEGF option together.

Fields: max-norm relative error <= 1e-10.  Cellular automaton: bit-exact.
"""
import numpy as np
import pytest

from oracle import ca as oca
from oracle import model as om
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10
# boluses: drug 1 at 0; drug 2 at 20; drug 3 at 0, 45 (between substep ends) and 100
TIMES = ((0.0,), (20.0,), (0.0, 45.0, 100.0))
AMTS = ((1.0,), (0.8,), (1.0, 0.7, 0.9))


def relerr(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def params(**kw):
    base = dict(cg_rtol=1e-15, init_rtol=1e-15, cg_maxit=20000, init_maxit=400, drug3=1)
    base.update(kw)
    return hca.default_params(**base)


def push(sim, s, names=("L", "K", "G1", "G2", "P", "Vc", "phi", "G3")):
    for name in names:
        sim.set_field(name, getattr(s, name))
    sim.set_step(s.step)


@pytest.fixture(scope="module")
def case32d():
    print("\n[case32d] 32^3, 8 Gaussians, seed 1, third drug", flush=True)
    tis = synth.make_tissue(32, 8, seed=1)
    op = OP.with_(drug3=1)
    s0 = om.init_state(tis.cell, tis.w, tis.seed, op)
    return tis, op, s0


def sim_of(tis, **kw):
    return hca.Simulation([(tis.cell, tis.w, tis.seed, (TIMES, AMTS))], params(**kw))


def test_init_has_zero_third_drug(case32d):
    tis, _, _ = case32d
    with sim_of(tis) as sim:
        assert not sim.field("G3").any()
    with sim_of(tis, drug3=0) as sim:
        with pytest.raises(RuntimeError):
            sim.field("G3")


@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 0.5)], ids=["be1", "cn3"])
@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_third_drug_field_matches_oracle(case32d, m, theta, precond):
    """The drug fields over four steps (boluses of the third drug at 0, 45
    and 100 min), restarting from the oracle's state each step."""
    print(f"\n[drug3] m {m} theta {theta} precond {precond}", flush=True)
    tis, op, s0 = case32d
    opm = op.with_(pde_substeps=m, pde_theta=theta)
    sched = om.Schedule(times=TIMES, amts=AMTS)
    s = s0
    with sim_of(tis, precond=precond, pde_substeps=m, pde_theta=theta) as sim:
        for n in range(4):
            push(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            K, G1, G2 = om.solve_fields(s, tis.w, sched, opm)
            G3 = om.solve_drug3(s, tis.w, sched, opm)
            assert G3.max() > 0.0
            for name, ref in (("K", K), ("G1", G1), ("G2", G2), ("G3", G3)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
            assert sim.stats()["cg_iters_drug3"] > 0
            s, _ = om.step(s, tis.w, sched, tis.seed, opm)


@pytest.mark.parametrize("seed", [0, 1])
def test_third_kill_trial_bit_exact(case32d, seed):
    tis, op, s0 = case32d
    rng = np.random.default_rng(40 + seed)
    shape = tis.cell.shape
    s = s0.copy()
    s.K = 5.0 + 15.0 * rng.random(shape)
    s.G1 = rng.random(shape) * 0.1
    s.G2 = rng.random(shape) * 0.1
    s.G3 = rng.random(shape) * 0.6
    s.phi = np.where(s.L == 1, rng.choice([0.3, 1.0, 1.2], size=shape), 0.0)
    s.step = int(rng.integers(0, 500))
    with sim_of(tis) as sim:
        push(sim, s)
        sim.run_phases(hca.PH_CA | hca.PH_STATS)
        Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, tis.w, s.K, s.G1, s.G2, s.phi, s.P, s.Vc,
                                                   s.step, tis.seed, op, s.G3)
        assert np.array_equal(sim.field("L"), Ln)
        assert np.array_equal(sim.field("phi"), phin)
        assert np.array_equal(sim.field("P"), Pn) and np.array_equal(sim.field("Vc"), Vn)
        st = sim.stats()
        assert (st["kills"], st["divisions"]) == (ev["kills"], ev["divisions"])
        # more kills than the two-drug automaton on the same state
        _, _, _, _, ev2, _, _ = oca.ca_update(s.L, tis.w, s.K, s.G1, s.G2, s.phi, s.P, s.Vc,
                                              s.step, tis.seed, op)
        assert ev["kills"] > ev2["kills"]


def test_third_drug_with_vegf_full_steps(case32d):
    """hca_step with both options (fields [K | G1 | G2 | G3 | V]) across a
    vessel update, against the oracle's step from the same state."""
    tis, _, _ = case32d
    op = OP.with_(drug3=1, vegf=1, V_high=3.0e-5, p_death=0.5, birth_per_V=0.05 / 3.0e-5)
    s = om.init_state(tis.cell, tis.w, tis.seed, op)
    s.step = 21
    sched = om.Schedule(times=TIMES, amts=AMTS)
    kw = dict(vegf=1, V_high=op.V_high, p_death=op.p_death, birth_per_V=op.birth_per_V)
    with sim_of(tis, **kw) as sim:
        for n in range(3):
            push(sim, s, ("L", "K", "G1", "G2", "P", "Vc", "phi", "G3", "V", "w"))
            sim.step(1)
            s, ev = om.step(s, None, sched, tis.seed, op)
            for name in ("K", "G1", "G2", "G3", "V"):
                assert relerr(sim.field(name), getattr(s, name)) <= FIELD_TOL, (n, name)
            assert np.array_equal(sim.field("L"), s.L), n
            assert np.array_equal(sim.field("w"), s.w), n
            st = sim.stats()
            assert (st["kills"], st["vessel_births"], st["vessel_deaths"]) == \
                (ev["kills"], ev["births"], ev["deaths"]), n
