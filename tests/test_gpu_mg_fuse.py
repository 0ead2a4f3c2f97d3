"""Level 0 of the multigrid with its three pre-sweeps + restriction and its
three post-sweeps each fused into one pass (mg_fuse = 1, the default)
against one kernel per sweep (mg_fuse = 0), through the C ABI.

The two compute the same V-cycle up to the rounding order of the neighbour
sums (FP32), so the flexible CG takes the same number of iterations (with
the geometric initial guess: the fitted one picks among candidates whose
residuals can tie to rounding, and a different pick may change a count by
one) and the
fields agree to the solve tolerance: <= 1e-12 relative in precision 64 (the
solves stop at 1e-10 residual from either preconditioner) and <= 1e-6 in
precision 32 (1e-8 floor).  The lattices cover even, odd, 2-D, thin,
single-cell and tile-straddling shapes; each field's solve is parity-tested
against the oracle elsewhere with the default (fused) path."""
import numpy as np
import pytest

from paper_2105_00448_amd import hca, synth

pytestmark = pytest.mark.gpu

SHAPES = [((48, 40, 36), 8, 3), ((37, 50, 29), 4, 4), ((1, 90, 77), 4, 5), ((33, 17, 65), 4, 6),
          ((5, 3, 130), 2, 8), ((1, 1, 1), 1, 9), ((2, 40, 2), 2, 10), ((70, 9, 20), 4, 11)]


def relerr(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape,ng,seed", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_fused_level0_smoothing_matches_per_sweep_kernels(shape, ng, seed, precision):
    print(f"\n[mg fuse] {shape} precision {precision}", flush=True)
    tis = synth.make_tissue(shape, ng, seed=seed)
    if not (tis.w > 0).any():
        tis.w.ravel()[0] = 1.0
        tis.cell.ravel()[0] = 0
    sched = synth.bolus_schedule([0, 2])
    reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
    out = {}
    for fuse in (0, 1):
        with hca.Simulation(reps, hca.default_params(precision=precision, mg_fuse=fuse, x0_extrapolate=2)) as sim:
            iters = []
            for _ in range(4):
                sim.step(1)
                iters.append(list(sim.stats()["cg_iters"]))
            out[fuse] = ({k: sim.field(k) for k in ("K", "G1", "G2", "L")}, iters)
    (f0, i0), (f1, i1) = out[0], out[1]
    assert i0 == i1
    tol = 1e-12 if precision == 64 else 1e-6
    for k in ("K", "G1", "G2"):
        assert relerr(f1[k], f0[k]) <= tol, k
    assert np.array_equal(f1["L"], f0["L"])


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape", [(48, 40, 36), (64, 64, 32), (32, 96, 16)], ids=str)
def test_fused_coarser_levels_match_per_sweep_kernels(shape, precision, monkeypatch):
    """Coarser levels whose cells are all full 2^k-cubes also smooth in fused
    passes (two stages before and after; by default only on levels of at
    least 2 M cells over all systems, here forced on every eligible level):
    the same iteration counts and fields as one kernel per sweep."""
    print(f"\n[mg fuse levels] {shape} precision {precision}", flush=True)
    tis = synth.make_tissue(shape, 8, seed=sum(shape))
    sched = synth.bolus_schedule([0, 2])
    reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
    out = {}
    for fuse in (0, 1):
        monkeypatch.setenv("HCA_FUSE_MIN_CELLS", "1")
        with hca.Simulation(reps, hca.default_params(precision=precision, mg_fuse=fuse, x0_extrapolate=2)) as sim:
            iters = []
            for _ in range(4):
                sim.step(1)
                iters.append(list(sim.stats()["cg_iters"]))
            out[fuse] = ({k: sim.field(k) for k in ("K", "G1", "G2")}, iters)
    monkeypatch.delenv("HCA_FUSE_MIN_CELLS")
    (f0, i0), (f1, i1) = out[0], out[1]
    assert i0 == i1
    tol = 1e-12 if precision == 64 else 1e-6
    for k in ("K", "G1", "G2"):
        assert relerr(f1[k], f0[k]) <= tol, k


def test_fused_path_in_a_batch_with_uneven_replicates():
    """A batch of replicates of different shapes (tile widths 16 and 32, one
    2-D) solved together with the fused passes: each replicate equals its own
    single-replicate context's fields to the solve tolerance."""
    cases = [synth.make_tissue(s, 4, seed=20 + i) for i, s in enumerate([(40, 36, 20), (12, 14, 30), (1, 50, 41)])]
    sched = synth.bolus_schedule([0])
    reps = [(t.cell, t.w, t.seed, (sched.times, sched.amts)) for t in cases]
    with hca.Simulation(reps, hca.default_params(mg_fuse=1, x0_extrapolate=2)) as sim:
        sim.step(3)
        got = [{k: sim.field(k, r) for k in ("K", "G1", "G2")} for r in range(len(reps))]
    for r, rep in enumerate(reps):
        with hca.Simulation([rep], hca.default_params(mg_fuse=0, x0_extrapolate=2)) as one:
            one.step(3)
            for k in ("K", "G1", "G2"):
                assert relerr(got[r][k], one.field(k)) <= 1e-12, (r, k)
