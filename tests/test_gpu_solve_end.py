"""The last CG iteration's x += alpha p of a step's solves is made by the ODE
kernel that follows them (it reads every voxel of the fields anyway); when
the phases run as separate calls, the solve makes it itself.  Both orders
must give the same state bit for bit: plain in both precisions, with θ-scheme
substeps (only the last substep's solve leaves its end to the ODE phase) and
with Newton steps on the oxygen uptake (none does), on one context of uneven
replicates with a drug-free control (the solver's scalars are indexed by
field and replicate).  The surrogate's kernel is covered in test_gpu_mlp.py.
"""
import numpy as np
import pytest

from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

NAMES = ("L", "K", "G1", "G2", "P", "Vc", "phi")
SPECS = [
    # (shape (nz, ny, nx), seed, dose schedule)
    ((10, 12, 9), 41, synth.bolus_schedule([0, 2])),
    ((1, 18, 21), 42, synth.bolus_schedule([1])),                               # 2-D slice
    ((8, 8, 8), 43, synth.DoseSchedule(times=((), ()), amts=((), ()))),        # drug-free
]


def replicates():
    out = []
    for shape, seed, sched in SPECS:
        t = synth.make_tissue(shape, 4, seed=seed)
        out.append((t.cell, t.w, t.seed, (sched.times, sched.amts)))
    return out


def assert_same(a, b, where):
    for r in range(len(SPECS)):
        for name in NAMES:
            np.testing.assert_array_equal(a.field(name, r), b.field(name, r),
                                          err_msg=f"{where} replicate {r} {name}")
        np.testing.assert_equal(a.stats(r), b.stats(r), err_msg=f"{where} replicate {r} stats")


@pytest.mark.parametrize("kw", [dict(precision=64), dict(precision=32),
                                dict(precision=64, pde_substeps=2),
                                dict(precision=64, o2_newton=1)],
                         ids=["fp64", "fp32", "substeps", "newton"])
def test_solve_end_in_the_ode_phase_is_the_separate_one(kw):
    print(f"\n[solve end] {kw}", flush=True)
    prm = hca.default_params(**kw)
    reps = replicates()
    with hca.Simulation(reps, prm) as a, hca.Simulation(reps, prm) as b:
        for n in range(4):
            a.step()
            b.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            b.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            assert_same(a, b, f"{kw} step {n}")
