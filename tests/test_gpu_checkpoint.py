"""Checkpoint and resume through the C ABI: a run continued from exported
states is bit-identical to the uninterrupted run (every field, the cell map,
the vessel map and the cumulative counts), whether it resumes in a new
context (hca_init_from_state) or rolls an existing one back
(hca_import_state); malformed states are rejected and leave the state as
it was."""
import numpy as np
import pytest

from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

FIELDS = ("L", "K", "G1", "G2", "P", "Vc", "phi", "w")


def cases(options):
    """Two uneven replicates (one a 2-D slice); with options, the third drug
    is dosed too."""
    out = []
    for shape, seed in (((14, 18, 16), 61), ((1, 30, 25), 62)):
        t = synth.make_tissue(shape, 4, seed=seed)
        if options:
            sched = ((0.0, 150.0), (0.0, 150.0), (30.0,)), ((1.0, 0.6), (1.0, 0.6), (1.0,))
        else:
            sched = ((0.0, 150.0), (0.0, 150.0)), ((1.0, 0.6), (1.0, 0.6))
        out.append((t.cell, t.w, t.seed, sched))
    return out


OPTIONS = dict(vegf=1, dv_min=60.0, drug3=1, pk_mm=1, pde_substeps=2, pde_theta=0.5, o2_newton=1)


def field_names(options):
    return FIELDS + (("V", "G3") if options else ())


def snapshot(sim, nrep, names):
    return [{k: sim.field(k, r) for k in names} for r in range(nrep)]


@pytest.mark.parametrize("options", [False, True], ids=["plain", "all-options"])
def test_resume_is_bit_identical(options):
    print(f"\n[checkpoint] options {options}", flush=True)
    reps = cases(options)
    params = hca.default_params(**(OPTIONS if options else {}))
    names = field_names(options)
    with hca.Simulation(reps, params) as full:
        full.step(20)
        want = snapshot(full, len(reps), names)
        want_stats = [full.stats(r) for r in range(len(reps))]
    with hca.Simulation(reps, params) as first:
        first.step(10)
        blobs = [first.export_state(r) for r in range(len(reps))]
        mid = snapshot(first, len(reps), names)
    # resumed in a new context; the replicates' maps come from the states
    resume_reps = [(None, None, seed, sched) for (_, _, seed, sched) in reps]
    with hca.Simulation(resume_reps, params, states=blobs) as sim:
        assert sim.stats()["step"] == 10
        for r in range(len(reps)):
            for k in names:
                assert np.array_equal(sim.field(k, r), mid[r][k]), (r, k)
        sim.step(10)
        for r in range(len(reps)):
            for k in names:
                assert np.array_equal(sim.field(k, r), want[r][k]), (r, k)
            st = sim.stats(r)
            for k in ("step", "total_divisions", "total_kills", "n_cancer", "n_vessel",
                      "total_births", "total_deaths"):
                assert st[k] == want_stats[r][k], (r, k)
        assert want_stats[0]["total_divisions"] > 0
        if options:
            assert sum(s["total_births"] + s["total_deaths"] for s in want_stats) > 0


def test_import_rolls_back_and_replays():
    reps = cases(False)
    with hca.Simulation(reps) as sim:
        sim.step(10)
        blobs = [sim.export_state(r) for r in range(len(reps))]
        sim.step(10)
        want = snapshot(sim, len(reps), FIELDS)
        sim.step(3)
        # a context of several replicates: every replicate back to step 10
        for r in range(len(reps)):
            if r == 0:
                with pytest.raises(hca.HcaError) as e:   # step 23 != 10 for replicate 0 alone
                    sim.import_state(blobs[0], 0)
                assert e.value.status == hca.E_INVALID
                sim.set_step(10)
            sim.import_state(blobs[r], r)
        sim.step(10)
        got = snapshot(sim, len(reps), FIELDS)
    for r in range(len(reps)):
        for k in FIELDS:
            assert np.array_equal(got[r][k], want[r][k]), (r, k)


def test_bad_states_are_rejected_and_change_nothing():
    reps = cases(False)
    with hca.Simulation(reps) as sim:
        sim.step(2)
        blob0 = sim.export_state(0)
        blob1 = sim.export_state(1)
        before = snapshot(sim, len(reps), FIELDS)

        def status(blob, rep):
            with pytest.raises(hca.HcaError) as e:
                sim.import_state(blob, rep)
            return e.value.status

        assert status(blob1, 0) == hca.E_INVALID           # other lattice and seed
        assert status(blob0[:-8], 0) == hca.E_RANGE        # truncated
        assert status(blob0[:50], 0) == hca.E_RANGE
        bad = blob0.copy()
        bad[0] ^= 1                                        # not a state blob
        assert status(bad, 0) == hca.E_INVALID
        bad = blob0.copy()
        bad[96] = 7                                        # cell code 7
        assert status(bad, 0) == hca.E_INVALID
        after = snapshot(sim, len(reps), FIELDS)
        for r in range(len(reps)):
            for k in FIELDS:
                assert np.array_equal(after[r][k], before[r][k]), (r, k)
        sim.step(1)                                        # the context still works
    # resume with a wrong seed, or states at different steps
    with hca.Simulation(reps) as a:
        a.step(1)
        b1 = [a.export_state(r) for r in range(len(reps))]
        a.step(1)
        b2 = [a.export_state(r) for r in range(len(reps))]
    resume = [(None, None, seed, sched) for (_, _, seed, sched) in reps]
    wrong_seed = [(None, None, seed + 1, sched) for (_, _, seed, sched) in reps]
    with pytest.raises(hca.HcaError) as e:
        hca.Simulation(wrong_seed, states=b1)
    assert e.value.status == hca.E_INVALID
    with pytest.raises(hca.HcaError) as e:
        hca.Simulation(resume, states=[b1[0], b2[1]])
    assert e.value.status == hca.E_INVALID


def test_state_without_the_second_guess_level_restarts_it():
    """A state exported with the geometric guess (x0_extrapolate = 2: one
    history level) imports into a context with the fitted guess (two levels):
    the missing level restarts from the first, and the run continues to the
    same fields (solves to 1e-15: the guess changes iteration counts, not the
    converged fields) and cell map."""
    reps = cases(False)
    tight = dict(cg_rtol=1e-15, init_rtol=1e-15, cg_maxit=20000, init_maxit=400)
    with hca.Simulation(reps, hca.default_params(x0_extrapolate=2, **tight)) as src:
        src.step(6)
        blobs = [src.export_state(r) for r in range(len(reps))]
    resume_reps = [(None, None, seed, sched) for (_, _, seed, sched) in reps]
    with hca.Simulation(resume_reps, hca.default_params(x0_extrapolate=3, **tight), states=blobs) as fit, \
            hca.Simulation(resume_reps, hca.default_params(x0_extrapolate=2, **tight), states=blobs) as geo:
        fit.step(6)
        geo.step(6)
        for r in range(len(reps)):
            assert np.array_equal(fit.field("L", r), geo.field("L", r)), r
            for k in ("K", "G1", "G2"):
                a, b = fit.field(k, r), geo.field(k, r)
                scale = np.abs(b).max()
                assert np.abs(a - b).max() <= 1e-10 * (scale if scale > 0 else 1.0), (r, k)
