"""Precision 32 (solved fields and solver arrays stored in FP32) against the
FP64 oracle, through the C ABI.

* Fields: max-norm relative error <= 1e-5.  The solves stop at a relative
  residual of 1e-8 (the FP32 floor); an FP32 prototype of the same CG on
  the 32^3 oxygen system measured 2e-6 there, and the solution rounded to
  FP32 is good to 6e-8.
* The inputs a precision-32 context holds are FP32 values: the oracle takes
  the same values (its state's K, G1, G2 rounded to FP32 and read back as
  FP64), so the ODE and the cellular automaton, which compute in FP64 from
  them, must match bit for bit (P, V_c to 1e-10 as in precision 64).
"""
import numpy as np
import pytest

from oracle import ca as oca
from oracle import model as om
from oracle import ode as oode
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10
SOLVED = ("K", "G1", "G2")


def relerr(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def params32(**kw):
    # the FP64 initialisation at the tolerances of the FP64 parity tests; the
    # FP32 solves stop at their 1e-8 floor
    base = dict(precision=32, cg_rtol=1e-15, init_rtol=1e-15, cg_maxit=20000, init_maxit=400)
    base.update(kw)
    return hca.default_params(**base)


def rounded(s):
    """The state as a precision-32 context holds it."""
    t = s.copy()
    for name in SOLVED:
        setattr(t, name, f32(getattr(s, name)))
    if t.G3 is not None:
        t.G3 = f32(t.G3)
    if t.V is not None:
        t.V = f32(t.V)
    return t


def push(sim, s, rep=0):
    for name in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
        sim.set_field(name, getattr(s, name), rep)
    sim.set_step(s.step)


@pytest.fixture(scope="module")
def case32():
    print("\n[fp32 case32] 32^3, 8 Gaussians, seed 1", flush=True)
    tis = synth.make_tissue(32, 8, seed=1)
    sched = synth.bolus_schedule([0])
    s0 = om.init_state(tis.cell, tis.w, tis.seed, OP)
    return tis, sched, s0


def sim_of(cases, **kw):
    reps = [(t.cell, t.w, t.seed, (s.times, s.amts)) for t, s in cases]
    return hca.Simulation(reps, params32(**kw))


def test_init_is_the_fp64_init_rounded(case32):
    tis, sched, s0 = case32
    with sim_of([(tis, sched)]) as sim:
        K = sim.field("K")
        assert np.array_equal(K, f32(K))              # stored in FP32
        assert relerr(K, s0.K) <= 1e-7                # the FP64 steady state, rounded once
        assert relerr(sim.field("P"), s0.P) <= TOL64  # cell state from the FP64 oxygen
        assert relerr(sim.field("Vc"), s0.Vc) <= TOL64
        assert np.array_equal(sim.field("phi"), s0.phi)
        assert not sim.field("G1").any()


@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_solves_within_1e5(case32, precond):
    tis, sched, s0 = case32
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = s0
    for _ in range(2):
        s, _ = om.step(s, tis.w, osched, tis.seed, OP)
    s = rounded(s)
    with sim_of([(tis, sched)], precond=precond) as sim:
        push(sim, s)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        ref = om.solve_fields(s, tis.w, osched, OP)
        for name, r in zip(SOLVED, ref):
            got = sim.field(name)
            err = relerr(got, r)
            print(f"[fp32 solve] precond {precond} {name}: {err:.2e}", flush=True)
            assert err <= TOL32, name
            assert np.array_equal(got, f32(got))
        st = sim.stats()
        assert all(i > 0 for i in st["cg_iters"])
        assert all(r <= 1.01e-8 for r in st["cg_relres"])


def test_ode_and_ca_bit_exact_on_shared_fp32_fields(case32):
    tis, sched, s0 = case32
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = s0
    for _ in range(3):
        s, _ = om.step(s, tis.w, osched, tis.seed, OP)
    K, G1, G2 = (f32(x) for x in om.solve_fields(s, tis.w, osched, OP))
    with sim_of([(tis, sched)]) as sim:
        push(sim, s)
        for name, v in (("K", K), ("G1", G1), ("G2", G2)):
            sim.set_field(name, v)
        sim.run_phases(hca.PH_ODE)
        P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, OP)
        assert relerr(sim.field("P"), P) <= TOL64
        assert relerr(sim.field("Vc"), Vc) <= TOL64
        assert np.array_equal(sim.field("phi"), phi)
        sim.set_field("P", P)
        sim.set_field("Vc", Vc)
        sim.set_field("phi", phi)
        sim.run_phases(hca.PH_CA | hca.PH_STATS)
        Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, tis.w, K, G1, G2, phi, P, Vc, s.step,
                                                   tis.seed, OP)
        assert np.array_equal(sim.field("L"), Ln)
        assert np.array_equal(sim.field("phi"), phin)
        assert np.array_equal(sim.field("P"), Pn)
        assert np.array_equal(sim.field("Vc"), Vn)
        st = sim.stats()
        for k in ("committed", "kills", "divisions", "nospace", "lost"):
            assert st[k] == ev[k], k
        assert ev["divisions"] > 0 and ev["kills"] > 0


@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_trajectory_10_steps_resynchronised(case32, precond):
    """Each step from the oracle's (FP32-rounded) state: solves <= 1e-5, then
    the ODE and the CA on the shared fields bit-exact."""
    tis, sched, s0 = case32
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = rounded(s0)
    worst = 0.0
    with sim_of([(tis, sched)], precond=precond) as sim:
        for n in range(10):
            push(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            ref = om.solve_fields(s, tis.w, osched, OP)
            for name, r in zip(SOLVED, ref):
                err = relerr(sim.field(name), r)
                worst = max(worst, err)
                assert err <= TOL32, (n, name)
            # shared fields for the cell update: the oracle's, rounded to FP32
            K, G1, G2 = (f32(x) for x in ref)
            for name, v in (("K", K), ("G1", G1), ("G2", G2)):
                sim.set_field(name, v)
            sim.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, OP)
            Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, tis.w, K, G1, G2, phi, P, Vc, s.step,
                                                       tis.seed, OP)
            assert np.array_equal(sim.field("L"), Ln), n
            assert np.array_equal(sim.field("phi"), phin), n
            assert relerr(sim.field("P"), Pn) <= TOL64
            assert relerr(sim.field("Vc"), Vn) <= TOL64
            s = om.State(Ln, K, G1, G2, Pn, Vn, phin, s.step + 1)
    print(f"[fp32 trajectory] precond {precond}: worst field error {worst:.2e}", flush=True)


@pytest.mark.parametrize("shape", [(9, 23, 17), (1, 40, 33), (2, 2, 130), (1, 1, 1)])
def test_ragged_and_batched(shape):
    """A ragged lattice alone and in a batch with a 20^3 lattice: solves
    <= 1e-5 against the oracle on each replicate."""
    tis = synth.make_tissue(shape, 4, seed=sum(shape))
    if not (tis.w > 0).any():
        tis.w.ravel()[0] = 1.0
        tis.cell.ravel()[0] = 0
    other = synth.make_tissue(20, 4, seed=77)
    sched = synth.bolus_schedule([0, 2])
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    cases = [(tis, sched), (other, sched)]
    states = [rounded(om.init_state(t.cell, t.w, t.seed, OP)) for t, _ in cases]
    for batch in (cases[:1], cases):
        with sim_of(batch) as sim:
            for n in range(2):
                for r in range(len(batch)):
                    push(sim, states[r], r)
                sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
                for r, (t, _) in enumerate(batch):
                    ref = om.solve_fields(states[r], t.w, osched, OP)
                    for name, x in zip(SOLVED, ref):
                        assert relerr(sim.field(name, r), x) <= TOL32, (shape, len(batch), n, r, name)
        # advance the oracle states for the next batch size's comparison
    del states


def test_every_option_within_1e5():
    """Third drug, VEGF with vessel updates, exact Michaelis-Menten, two
    Crank-Nicolson substeps and a Newton step, precision 32: each step's
    fields (K, G1, G2, G3, V) <= 1e-5 against the oracle from the oracle's
    FP32-rounded state, over four steps across a vessel update."""
    tis = synth.make_tissue((9, 23, 17), 4, seed=3)
    sched = synth.DoseSchedule(times=((0.0, 60.0), (0.0,), (30.0,)), amts=((1.0, 0.5), (0.8,), (1.0,)))
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    opts = dict(drug3=1, vegf=1, dv_min=60.0, pk_mm=1, pde_substeps=2, pde_theta=0.5, o2_newton=1)
    OPo = OP.with_(**opts)
    s = om.init_state(tis.cell, tis.w, tis.seed, OPo)
    reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
    with hca.Simulation(reps, params32(**opts)) as sim:
        for n in range(4):
            s = rounded(s)
            push(sim, s)
            sim.set_field("G3", s.G3)
            sim.set_field("V", s.V)
            sim.set_field("w", s.w)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS | hca.PH_VEGF)
            s2, _ = om.step(s, tis.w, osched, tis.seed, OPo)
            for name in ("K", "G1", "G2", "G3", "V"):
                err = relerr(sim.field(name), getattr(s2, name))
                assert err <= TOL32, (n, name, err)
            s = s2


def test_checkpoint_resume_bit_identical_in_fp32():
    tis = synth.make_tissue((14, 18, 16), 4, seed=61)
    sched = synth.bolus_schedule([0, 5])
    reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
    p = params32()
    with hca.Simulation(reps, p) as full:
        full.step(12)
        want = {k: full.field(k) for k in ("L", "K", "G1", "G2", "P", "Vc", "phi")}
    with hca.Simulation(reps, p) as first:
        first.step(6)
        blob = first.export_state(0)
    with hca.Simulation([(None, None, tis.seed, (sched.times, sched.amts))], p, states=[blob]) as sim:
        sim.step(6)
        for k, v in want.items():
            assert np.array_equal(sim.field(k), v), k
