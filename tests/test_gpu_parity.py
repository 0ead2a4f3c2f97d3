"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Fields: max-norm relative error <= 1e-10 (FP64 solves taken to a relative
residual of 1e-13 here, so the solver error stays far below the bar).
Cellular automaton and everything integer: bit-exact on shared inputs.
"""
import numpy as np
import pytest

from oracle import ca as oca
from oracle import model as om
from oracle import ode as oode
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10


def parity_params(**kw):
    base = dict(cg_rtol=1e-15, init_rtol=1e-15, cg_maxit=20000, init_maxit=400)
    base.update(kw)
    return hca.default_params(**base)


def relerr(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def oracle_sched(sched):
    return om.Schedule(times=sched.times, amts=sched.amts)


def make_sim(tissues_scheds, **kw):
    reps = [(t.cell, t.w, t.seed, (s.times, s.amts)) for t, s in tissues_scheds]
    return hca.Simulation(reps, parity_params(**kw))


def push_state(sim, s, rep=0):
    for name in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
        sim.set_field(name, getattr(s, name), rep)
    sim.set_step(s.step)


@pytest.fixture(scope="module")
def case32():
    print("\n[case32] 32^3, 8 Gaussians, seed 1", flush=True)
    tis = synth.make_tissue(32, 8, seed=1)
    sched = synth.bolus_schedule([0])
    s0 = om.init_state(tis.cell, tis.w, tis.seed, OP)
    return tis, sched, s0


def test_init_matches_oracle(case32):
    tis, sched, s0 = case32
    with make_sim([(tis, sched)]) as sim:
        assert np.array_equal(sim.field("L"), s0.L)
        assert relerr(sim.field("K"), s0.K) <= FIELD_TOL
        assert relerr(sim.field("P"), s0.P) <= FIELD_TOL
        assert relerr(sim.field("Vc"), s0.Vc) <= FIELD_TOL
        assert np.array_equal(sim.field("phi"), s0.phi)      # Philox uniforms, exact
        assert not sim.field("G1").any() and not sim.field("G2").any()
        st = sim.stats()
        assert st["n_cancer"] == np.count_nonzero(s0.L == 1)
        assert st["n_vessel"] == np.count_nonzero(tis.w > 0)


PRECONDS = pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
# solver variants: Jacobi; multigrid with the default one-workgroup coarse
# solve (levels up to 4096 cells); multigrid with more multi-workgroup levels
# (one-workgroup solve from 64 cells)
SOLVERS = pytest.mark.parametrize(
    "solver_kw", [dict(precond=0), dict(precond=1), dict(precond=1, mg_coarse_max=64)],
    ids=["jacobi", "multigrid", "multigrid-coarse64"])


@SOLVERS
def test_solves_match_oracle_exact_solution(case32, solver_kw):
    tis, sched, s0 = case32
    osched = oracle_sched(sched)
    # a state with drug already in the tissue: two oracle steps from init
    s = s0
    for _ in range(2):
        s, _ = om.step(s, tis.w, osched, tis.seed, OP)
    with make_sim([(tis, sched)], **solver_kw) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        K, G1, G2 = om.solve_fields(s, tis.w, osched, OP)
        assert relerr(sim.field("K"), K) <= FIELD_TOL
        assert relerr(sim.field("G1"), G1) <= FIELD_TOL
        assert relerr(sim.field("G2"), G2) <= FIELD_TOL
        it = sim.stats()["cg_iters"]
        assert all(i > 0 for i in it)


@pytest.mark.parametrize("m,theta", [(3, 1.0), (3, 0.5), (2, 0.7)], ids=["be3", "cn3", "theta07x2"])
@pytest.mark.parametrize("precond", [0, 1], ids=["jacobi", "multigrid"])
def test_field_substeps_match_oracle(case32, m, theta, precond):
    """The fields advanced in m theta-scheme substeps per coupled step (doses
    on and between substep boundaries), against the oracle over two steps;
    the steady-oxygen initialisation runs with the theta-scaled system."""
    print(f"\n[substeps] m {m} theta {theta} precond {precond}", flush=True)
    tis, _, s0 = case32
    sched = synth.DoseSchedule(times=((10.0, 45.0), (20.0,)), amts=((1.0, 0.5), (0.8,)))
    osched = oracle_sched(sched)
    OPm = OP.with_(pde_substeps=m, pde_theta=theta)
    with make_sim([(tis, sched)], precond=precond, pde_substeps=m, pde_theta=theta) as sim:
        assert relerr(sim.field("K"), s0.K) <= FIELD_TOL
        s = s0
        for n in range(2):
            push_state(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            K, G1, G2 = om.solve_fields(s, tis.w, osched, OPm)
            for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
            s, _ = om.step(s, tis.w, osched, tis.seed, OPm)
        it = sim.stats()["cg_iters"]
        assert all(i > 0 for i in it)


@pytest.mark.parametrize("m,theta,newton", [(1, 1.0, 3), (3, 0.5, 2)], ids=["be1-newton3", "cn3-newton2"])
def test_newton_oxygen_matches_oracle(case32, m, theta, newton):
    """Newton steps on the oxygen uptake at the new value after each
    linearised substep, against the oracle's, over two steps."""
    print(f"\n[newton] m {m} theta {theta} newton {newton}", flush=True)
    tis, sched, s0 = case32
    osched = oracle_sched(sched)
    OPn = OP.with_(pde_substeps=m, pde_theta=theta, o2_newton=newton)
    with make_sim([(tis, sched)], pde_substeps=m, pde_theta=theta, o2_newton=newton) as sim:
        s = s0
        for n in range(2):
            push_state(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            K, G1, G2 = om.solve_fields(s, tis.w, osched, OPn)
            for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
            s, _ = om.step(s, tis.w, osched, tis.seed, OPn)


@pytest.mark.parametrize("amt", [60.0, 2.0e4], ids=["halley", "log-newton"])
@pytest.mark.parametrize("m,theta", [(1, 1.0), (3, 0.5)], ids=["be1", "cn3"])
def test_michaelis_menten_plasma_matches_oracle(case32, amt, m, theta):
    """Fluorouracil plasma levels from the exact Michaelis-Menten decay
    (Lambert W; a bolus of 60 ug/mL takes the Halley branch, 2e4 ug/mL the
    large-argument branch), seen through the drug-2 field over two steps."""
    print(f"\n[mm] amount {amt} m {m} theta {theta}", flush=True)
    tis, _, s0 = case32
    sched = synth.DoseSchedule(times=((0.0,), (0.0, 45.0)), amts=((1.0,), (amt, 0.5 * amt)))
    osched = oracle_sched(sched)
    OPm = OP.with_(pde_substeps=m, pde_theta=theta, pk_mm=1)
    with make_sim([(tis, sched)], pde_substeps=m, pde_theta=theta, pk_mm=1) as sim:
        s = s0
        for n in range(2):
            push_state(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            K, G1, G2 = om.solve_fields(s, tis.w, osched, OPm)
            assert G2.max() > 0.0
            for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
            s, _ = om.step(s, tis.w, osched, tis.seed, OPm)


def test_ode_matches_oracle(case32):
    tis, sched, s0 = case32
    rng = np.random.default_rng(2)
    s = s0.copy()
    s.K = s0.K * (0.5 + rng.random(s0.K.shape))        # off the steady state
    s.Vc = s0.Vc * (0.5 + rng.random(s0.K.shape))
    s.Vc[s.L == 0] = 0.0
    with make_sim([(tis, sched)]) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_ODE)
        P, Vc, phi = oode.ode_step(s.L, s.K, s.P, s.Vc, s.phi, OP)
        assert relerr(sim.field("P"), P) <= FIELD_TOL
        assert relerr(sim.field("Vc"), Vc) <= FIELD_TOL
        assert np.array_equal(sim.field("phi"), phi)    # same rounding, no contraction


def random_ca_state(tis, rng):
    shape = tis.cell.shape
    L = tis.cell.copy()
    K = 5.0 + 15.0 * rng.random(shape)
    K[rng.random(shape) < 0.3] = 12.5                # exact ties
    G1 = rng.random(shape) * 0.4
    G2 = rng.random(shape) * 0.2
    phi = np.where(L == 1, rng.choice([0.3, 0.99, 1.0, 1.2, 1.2, 1.7], size=shape), 0.0)
    P = np.where(L != 0, rng.random(shape), 0.0)
    Vc = np.where(L != 0, rng.random(shape), 0.0)
    return om.State(L, K, G1, G2, P, Vc, phi, step=int(rng.integers(0, 1000)))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ca_bit_exact_on_shared_fields(case32, seed):
    tis, sched, _ = case32
    rng = np.random.default_rng(10 + seed)
    s = random_ca_state(tis, rng)
    with make_sim([(tis, sched)]) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_CA | hca.PH_STATS)
        Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, tis.w, s.K, s.G1, s.G2, s.phi, s.P, s.Vc,
                                                   s.step, tis.seed, OP)
        assert np.array_equal(sim.field("L"), Ln)
        assert np.array_equal(sim.field("phi"), phin)
        assert np.array_equal(sim.field("P"), Pn)
        assert np.array_equal(sim.field("Vc"), Vn)
        st = sim.stats()
        for k in ("committed", "kills", "divisions", "nospace", "lost"):
            assert st[k] == ev[k], k
        assert ev["divisions"] > 10 and ev["lost"] > 0 and ev["kills"] > 10


@PRECONDS
def test_trajectory_20_steps_resynchronised(case32, precond):
    """32^3 trajectory: each step's solves and ODE vs the oracle at the
    field tolerance, the CA bit-exact on the shared fields; the GPU restarts
    every step from the oracle's state."""
    tis, sched, s0 = case32
    osched = oracle_sched(sched)
    s = s0
    total_div = total_kill = 0
    with make_sim([(tis, sched)], precond=precond) as sim:
        for n in range(20):
            push_state(sim, s)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            K, G1, G2 = om.solve_fields(s, tis.w, osched, OP)
            for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
                assert relerr(sim.field(name), ref) <= FIELD_TOL, (n, name)
            # shared fields for the cell update
            sim.set_field("K", K)
            sim.set_field("G1", G1)
            sim.set_field("G2", G2)
            sim.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, OP)
            Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, tis.w, K, G1, G2, phi, P, Vc, s.step,
                                                       tis.seed, OP)
            assert np.array_equal(sim.field("L"), Ln), n
            assert np.array_equal(sim.field("phi"), phin), n
            assert relerr(sim.field("P"), Pn) <= FIELD_TOL
            assert relerr(sim.field("Vc"), Vn) <= FIELD_TOL
            st = sim.stats()
            assert st["step"] == n + 1
            assert (st["divisions"], st["kills"]) == (ev["divisions"], ev["kills"])
            total_div += ev["divisions"]
            total_kill += ev["kills"]
            s = om.State(Ln, K, G1, G2, Pn, Vn, phin, s.step + 1)
    assert total_div > 0 and total_kill > 0


@PRECONDS
def test_consecutive_steps_match_oracle(case32, precond):
    """Full steps in a row, nothing pushed between them, against the oracle's
    trajectory: the fields but oxygen keep their c and multigrid data from
    one step to the next, so this is where a stale operator would show.
    After two steps the vessel map changes (some vessels' weights doubled,
    some removed), which must rebuild them.  Fields within the field
    tolerance of the oracle's at every step, the cell map bit for bit."""
    tis, sched, s0 = case32
    osched = oracle_sched(sched)
    w = tis.w.copy()
    ves = np.flatnonzero(w.ravel() > 0)
    w2 = w.copy()
    w2.ravel()[ves[::3]] *= 2.0
    w2.ravel()[ves[1::7]] = 0.0
    s = s0
    with make_sim([(tis, sched)], precond=precond) as sim:
        for n in range(4):
            if n == 2:
                w = w2
                sim.set_field("w", w)
            sim.step()
            s, _ = om.step(s, w, osched, tis.seed, OP)
            for name in ("K", "G1", "G2", "P", "Vc", "phi"):
                assert relerr(sim.field(name), getattr(s, name)) <= FIELD_TOL, (n, name)
            assert np.array_equal(sim.field("L"), s.L), n
        assert sim.stats()["step"] == 4


@SOLVERS
@pytest.mark.parametrize("shape", [(9, 23, 17), (1, 40, 33), (70, 5, 5), (2, 2, 130), (1, 1, 1),
                                   (3, 1, 2)])
def test_ragged_lattices(shape, solver_kw):
    print(f"\n[ragged] shape {shape} solver {solver_kw}", flush=True)
    tis = synth.make_tissue(shape, 4, seed=sum(shape))
    if not (tis.w > 0).any():
        tis.w.ravel()[0] = 1.0
        tis.cell.ravel()[0] = 0
    sched = synth.bolus_schedule([0, 2])
    osched = oracle_sched(sched)
    s = om.init_state(tis.cell, tis.w, tis.seed, OP)
    with make_sim([(tis, sched)], **solver_kw) as sim:
        assert relerr(sim.field("K"), s.K) <= FIELD_TOL
        for n in range(4):
            push_state(sim, s)
            sim.run_phases(hca.PH_ALL)
            s2, ev = om.step(s, tis.w, osched, tis.seed, OP)
            for name in ("K", "G1", "G2", "P", "Vc"):
                assert relerr(sim.field(name), getattr(s2, name)) <= FIELD_TOL, (n, name)
            # CA on the oracle's fields: bit-exact
            push_state(sim, s)
            K, G1, G2 = om.solve_fields(s, tis.w, osched, OP)
            P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, OP)
            for name, v in (("K", K), ("G1", G1), ("G2", G2), ("P", P), ("Vc", Vc), ("phi", phi)):
                sim.set_field(name, v)
            sim.run_phases(hca.PH_CA)
            assert np.array_equal(sim.field("L"), s2.L)
            assert np.array_equal(sim.field("phi"), s2.phi)
            s = s2


@PRECONDS
def test_batched_replicates_equal_single_runs(precond):
    specs = [((20, 24, 28), 11, [0]), ((17, 17, 17), 12, [1]), ((8, 40, 31), 13, []),
             ((1, 33, 35), 14, [0])]
    cases = []
    for shape, seed, days in specs:
        t = synth.make_tissue(shape, 4, seed=seed)
        cases.append((t, synth.bolus_schedule(days)))
    kw = dict(cg_rtol=1e-10, init_rtol=1e-10, precond=precond)
    with make_sim(cases, **kw) as batch:
        batch.step(4)
        for r, case in enumerate(cases):
            with make_sim([case], **kw) as single:
                single.step(4)
                for name in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
                    assert np.array_equal(batch.field(name, r), single.field(name)), (r, name)
                assert batch.stats(r)["total_divisions"] == single.stats()["total_divisions"]


def test_runs_are_deterministic(case32):
    tis, sched, _ = case32
    out = []
    for _ in range(2):
        with make_sim([(tis, sched)], cg_rtol=1e-10, init_rtol=1e-10) as sim:
            sim.step(3)
            out.append([sim.field(n) for n in ("L", "K", "G1", "phi", "Vc")])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@PRECONDS
def test_graph_replay_equals_direct_launches(case32, precond):
    """CG iterations replayed from a captured HIP graph (many replays, with
    eager start/setup/CA work and host polls between them) give bit-identical
    fields to direct launches; also after a context's graph has been reused
    across several solves of different lengths."""
    tis, sched, _ = case32
    out = []
    for graphs in (0, 1):
        with make_sim([(tis, sched)], cg_rtol=1e-10, init_rtol=1e-10, precond=precond,
                      graphs=graphs) as sim:
            fields = []
            for _ in range(4):
                sim.step(1)
                fields.append([sim.field(n) for n in ("L", "K", "G1", "G2", "phi", "P", "Vc")])
            out.append(fields)
    for fa, fb in zip(*out):
        for a, b in zip(fa, fb):
            assert np.array_equal(a, b)


def test_autotuned_tiles_agree_with_heuristic_tiles(case32):
    """The tile autotuner only changes the tiling (and so the order of the
    dot-product partial sums): solves at rel. residual 1e-15 agree to
    rounding and the cellular automaton takes the same decisions."""
    tis, sched, _ = case32
    with make_sim([(tis, sched)], autotune=1) as a, make_sim([(tis, sched)], autotune=0) as b:
        tx, ty, tz = a.tile_shape()
        assert tx in (16, 32, 64) and tx * ty == 256 and 1 <= tz <= 16
        assert b.tile_shape() == (32, 8, b.tile_shape()[2])   # heuristic: tx from nx = 32
        a.step(3)
        b.step(3)
        assert np.array_equal(a.field("L"), b.field("L"))
        for n in ("K", "G1", "G2", "P", "Vc", "phi"):
            assert relerr(a.field(n), b.field(n)) <= 1e-12, n


@pytest.mark.parametrize("coarse_max", [64, 512, 4096])
@pytest.mark.parametrize("shape", [(32, 32, 32), (23, 17, 9), (40, 33, 1)], ids=str)
def test_multigrid_keeps_iterations_low(shape, coarse_max):
    """The V-cycle is only a preconditioner (parity cannot see a weak one), so
    its quality is pinned by iteration counts: at rel. residual 1e-10 every
    field converges in at most 14 flexible-CG iterations per step, on even,
    odd (ragged aggregates at every level) and 2-D lattices."""
    print(f"\n[mg iterations] {shape} coarse_max {coarse_max}", flush=True)
    tis = synth.make_tissue(shape, 6, seed=3)
    sched = synth.bolus_schedule([0])
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))],
                        hca.default_params(mg_coarse_max=coarse_max)) as sim:
        for _ in range(3):
            sim.step(1)
            it = sim.stats()["cg_iters"]
            assert max(it) <= 14, it


def test_error_paths_on_device(case32):
    tis, sched, _ = case32
    with make_sim([(tis, sched)], cg_rtol=1e-10, init_rtol=1e-10) as sim:
        bad = tis.cell.copy()
        bad[tis.w > 0] = 1
        with pytest.raises(hca.HcaError) as e:
            sim.set_field("L", bad)
        assert e.value.status == hca.E_INVALID
        with pytest.raises(hca.HcaError) as e:
            sim.field("K", rep=3)
        assert e.value.status == hca.E_RANGE
        sim.step(1)                 # context still usable
        K = sim.field("K")
        K[5, 5, 5] = np.nan
        sim.set_field("K", K)
        with pytest.raises(hca.HcaError) as e:
            sim.step(1)
        assert e.value.status in (hca.E_NONFINITE, hca.E_NOCONV)
        with pytest.raises(hca.HcaError) as e:
            sim.step(1)             # failed context refuses further steps
        assert e.value.status == hca.E_INVALID
        assert sim.field("L").shape == tis.cell.shape   # but still reads
    with pytest.raises(hca.HcaError) as e:
        make_sim([(tis, sched)], cg_rtol=1e-12, cg_maxit=2, init_rtol=1e-10)
    assert e.value.status == hca.E_NOCONV


def test_initial_guess_modes_agree(case32):
    """The solves' initial guess (plain, linear, geometric extrapolation, the
    least-squares fit over the two previous solutions) changes the iteration
    counts, not the converged fields: five full steps from the same state
    with boluses agree to the field tolerance, and once the plasma decays the
    geometric guess needs fewer drug iterations than the plain one and the
    fit no more than the geometric one."""
    tis, _, _ = case32
    sched = synth.DoseSchedule(times=((0.0,), (0.0, 60.0)), amts=((1.0,), (1.0, 0.5)))
    out, iters = {}, {}
    for mode in (0, 1, 2, 3):
        with make_sim([(tis, sched)], x0_extrapolate=mode) as sim:
            its = []
            for _ in range(5):
                sim.step(1)
                its.append(sim.stats()["cg_iters"])
            out[mode] = {n: sim.field(n) for n in ("K", "G1", "G2", "P", "Vc", "L")}
            iters[mode] = np.array(its)
    for mode in (1, 2, 3):
        for name in ("K", "G1", "G2", "P", "Vc"):
            assert relerr(out[mode][name], out[0][name]) <= FIELD_TOL, (mode, name)
        assert np.array_equal(out[mode]["L"], out[0]["L"]), mode
    # at the working tolerance, once the plasma decays (steps 6..12 after a
    # single bolus) the geometric guess saves drug iterations
    one = synth.bolus_schedule([0])
    for mode in (0, 2, 3):
        with make_sim([(tis, one)], x0_extrapolate=mode, cg_rtol=1e-10, init_rtol=1e-10) as sim:
            its = []
            for _ in range(12):
                sim.step(1)
                its.append(sim.stats()["cg_iters"])
            iters[mode] = np.array(its)
    assert iters[2][6:, 1:].sum() < iters[0][6:, 1:].sum(), (iters[0], iters[2])
    assert iters[3][6:, 1:].sum() <= iters[2][6:, 1:].sum(), (iters[2], iters[3])


@pytest.mark.parametrize("theta", [1.0, 0.5], ids=["be", "cn"])
def test_negative_oxygen_matches_oracle(case32, theta):
    """A state with oxygen below zero in places (what a Crank-Nicolson-type
    substep's oscillation can leave): the solves with the uptake continued by
    its tangent below 0, and the ODEs seeing max(K, 0), against the oracle."""
    tis, sched, s0 = case32
    osched = oracle_sched(sched)
    rng = np.random.default_rng(21)
    s = s0.copy()
    s.K = s0.K - 15.0 * (rng.random(s0.K.shape) < 0.2)         # some below -K1
    assert (s.K < 0.0).any() and (s.K < -OP.K1).any()
    op = OP.with_(pde_substeps=2, pde_theta=theta)
    with make_sim([(tis, sched)], pde_substeps=2, pde_theta=theta) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        K, G1, G2 = om.solve_fields(s, tis.w, osched, op)
        for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
            assert relerr(sim.field(name), ref) <= FIELD_TOL, name
        push_state(sim, s)
        sim.run_phases(hca.PH_ODE)
        P, Vc, phi = oode.ode_step(s.L, s.K, s.P, s.Vc, s.phi, op)
        assert relerr(sim.field("P"), P) <= FIELD_TOL
        assert relerr(sim.field("Vc"), Vc) <= FIELD_TOL
        assert np.array_equal(sim.field("phi"), phi)


@pytest.mark.parametrize("scale", [1e-60, 1e-120], ids=["1e-60", "1e-120"])
def test_tiny_drug_fields_match_oracle(case32, scale):
    """Drug fields far below FP32's range (long after the last dose): the
    multigrid's FP32 residual is scaled by a power of two per system, so the
    solves still converge and match the oracle."""
    tis, _, s0 = case32
    sched = synth.DoseSchedule(times=((), ()), amts=((), ()))
    osched = oracle_sched(sched)
    rng = np.random.default_rng(33)
    s = s0.copy()
    s.G1 = scale * rng.random(s0.K.shape)
    s.G2 = scale * 1e-3 * rng.random(s0.K.shape)
    with make_sim([(tis, sched)]) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        K, G1, G2 = om.solve_fields(s, tis.w, osched, OP)
        for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
            assert relerr(sim.field(name), ref) <= FIELD_TOL, name
        assert min(sim.stats()["cg_iters"][1:]) > 0


def test_negligible_drug_fields_count_as_solved(case32):
    """A drug field so small that its squared norms would leave FP64's normal
    range (||b||^2 < 1e-280) is left at its initial guess without error."""
    tis, _, s0 = case32
    sched = synth.DoseSchedule(times=((), ()), amts=((), ()))
    s = s0.copy()
    s.G1 = np.full(s0.K.shape, 1e-200)
    s.G2 = np.full(s0.K.shape, 1e-300)
    with make_sim([(tis, sched)]) as sim:
        push_state(sim, s)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        st = sim.stats()
        assert st["cg_iters"][1:] == [0, 0]
        for name in ("G1", "G2"):
            g = sim.field(name)
            assert np.isfinite(g).all() and np.abs(g).max() <= 1e-199


def test_long_run_past_the_last_dose(case32):
    """700 steps after a single bolus (the drug fields decay through FP32's
    range and towards FP64's): every solve converges and the state stays
    finite."""
    tis, sched, _ = case32
    with make_sim([(tis, sched)], cg_rtol=1e-10, init_rtol=1e-10) as sim:
        for _ in range(7):
            sim.step(100)
        st = sim.stats()
        assert st["step"] == 700 and not st["nonfinite"]
        g2 = sim.field("G2")
        assert np.isfinite(g2).all() and 0.0 < np.abs(g2).max() < 1e-30


# ---- a batched context against the oracle, replicate by replicate -----------------

BATCH_SPECS = [
    # (shape (nz, ny, nx), seed, dose schedule)
    ((12, 10, 9), 31, synth.bolus_schedule([0])),
    ((1, 20, 17), 32, synth.bolus_schedule([0, 2])),                   # 2-D slice
    ((16, 16, 16), 33, synth.DoseSchedule(times=((), ()), amts=((), ()))),   # drug-free control
    ((9, 23, 17), 34, synth.DoseSchedule(times=((30.0,), (30.0,)), amts=((1.3,), (0.6,)))),
    ((24, 8, 13), 35, synth.bolus_schedule([0, 2], amount=0.7)),
]


@PRECONDS
def test_batched_context_matches_oracle_per_replicate(precond):
    """One context holding five uneven replicates (incl. a 2-D slice and a
    drug-free control) against the oracle's step of each replicate on its
    own: every step restarts all replicates from the oracle's states; the
    batched solves <= 1e-10 per replicate; the ODE and CA on the shared
    fields bit-exact in L and phi (P, V_c <= 1e-10) with the same events."""
    cases = []
    for shape, seed, sched in BATCH_SPECS:
        t = synth.make_tissue(shape, 4, seed=seed)
        assert (t.w > 0).any()
        cases.append((t, sched))
    states = [om.init_state(t.cell, t.w, t.seed, OP) for t, _ in cases]
    totals = dict(divisions=0, kills=0)
    with make_sim(cases, precond=precond) as sim:
        for r, s in enumerate(states):
            assert relerr(sim.field("K", r), s.K) <= FIELD_TOL, r
            assert np.array_equal(sim.field("phi", r), s.phi), r
        for n in range(4):
            print(f"[batched vs oracle] precond {precond} step {n}", flush=True)
            for r, s in enumerate(states):
                push_state(sim, s, r)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            solved = []
            for r, ((t, sched), s) in enumerate(zip(cases, states)):
                K, G1, G2 = om.solve_fields(s, t.w, oracle_sched(sched), OP)
                for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
                    assert relerr(sim.field(name, r), ref) <= FIELD_TOL, (n, r, name)
                if r == 2:
                    assert not sim.field("G1", r).any() and not sim.field("G2", r).any()
                solved.append((K, G1, G2))
                for name, v in (("K", K), ("G1", G1), ("G2", G2)):
                    sim.set_field(name, v, r)
            sim.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            nxt = []
            for r, ((t, sched), s, (K, G1, G2)) in enumerate(zip(cases, states, solved)):
                P, Vc, phi = oode.ode_step(s.L, K, s.P, s.Vc, s.phi, OP)
                Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s.L, t.w, K, G1, G2, phi, P, Vc,
                                                           s.step, t.seed, OP)
                assert np.array_equal(sim.field("L", r), Ln), (n, r)
                assert np.array_equal(sim.field("phi", r), phin), (n, r)
                assert relerr(sim.field("P", r), Pn) <= FIELD_TOL, (n, r)
                assert relerr(sim.field("Vc", r), Vn) <= FIELD_TOL, (n, r)
                st = sim.stats(r)
                assert st["step"] == n + 1
                for k in ("committed", "kills", "divisions", "nospace", "lost"):
                    assert st[k] == ev[k], (n, r, k)
                totals["divisions"] += ev["divisions"]
                totals["kills"] += ev["kills"]
                if r == 2:
                    assert ev["kills"] == 0
                nxt.append(om.State(Ln, K, G1, G2, Pn, Vn, phin, s.step + 1))
            states = nxt
    assert totals["divisions"] > 0 and totals["kills"] > 0, totals


# ---- a lattice with three multi-workgroup multigrid levels --------------------------

@pytest.mark.slow
def test_96cube_three_global_mg_levels_match_oracle():
    """96^3 (32 Gaussians, ~86 % occupied) with the default one-workgroup
    coarse solve from 4096 cells: the V-cycle smooths 96^3, 48^3 and 24^3 with
    the multi-workgroup kernels before the 12^3 coarse solve.  Steady-oxygen
    init and one step's solves <= 1e-10 against the oracle, then the ODE and
    the CA on the shared fields bit-exact."""
    print("\n[96^3] oracle init (about 30 s)", flush=True)
    tis = synth.make_tissue(96, 32, seed=5)
    sched = synth.bolus_schedule([0])
    osched = oracle_sched(sched)
    s0 = om.init_state(tis.cell, tis.w, tis.seed, OP)
    with make_sim([(tis, sched)]) as sim:
        assert relerr(sim.field("K"), s0.K) <= FIELD_TOL
        assert np.array_equal(sim.field("phi"), s0.phi)
        sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        print("[96^3] oracle solves (about 30 s)", flush=True)
        K, G1, G2 = om.solve_fields(s0, tis.w, osched, OP)
        for name, ref in (("K", K), ("G1", G1), ("G2", G2)):
            err = relerr(sim.field(name), ref)
            print(f"[96^3] {name} rel. err {err:.2e}", flush=True)
            assert err <= FIELD_TOL, name
        for name, v in (("K", K), ("G1", G1), ("G2", G2)):
            sim.set_field(name, v)
        sim.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS)
        P, Vc, phi = oode.ode_step(s0.L, K, s0.P, s0.Vc, s0.phi, OP)
        Ln, phin, Pn, Vn, ev, _, _ = oca.ca_update(s0.L, tis.w, K, G1, G2, phi, P, Vc, 0,
                                                   tis.seed, OP)
        assert np.array_equal(sim.field("L"), Ln)
        assert np.array_equal(sim.field("phi"), phin)
        assert relerr(sim.field("P"), Pn) <= FIELD_TOL
        assert relerr(sim.field("Vc"), Vn) <= FIELD_TOL
        st = sim.stats()
        for k in ("committed", "kills", "divisions", "nospace", "lost"):
            assert st[k] == ev[k], k
        assert ev["divisions"] > 100 and ev["kills"] > 100
