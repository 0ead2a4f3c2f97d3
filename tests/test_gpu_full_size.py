"""The headline workload at its full size and in the launch configuration
that bench.py times: four replicates of a 384^3 lattice in one context
(512-Gaussian density, Philox seeds 5000-5003, a bolus of both drugs at step
0, default parameters: FP64 multigrid-preconditioned CG to relative residual
1e-10, captured iterations replayed as HIP graphs, the solves' last update
made inside the ODE kernel).  After two steps, one more coupled step is
checked against the oracle wherever the oracle can follow it at this size
(its full solves and its whole-lattice CA would take hours on one core):

* the solves (Eqs. (oxygen), (chemo)): every field's true relative residual,
  with the oracle's own systems (`o2_system`, `drug_system` built from the
  state before the step, the plasma levels from its PK) and its operator,
  below the stopping tolerance with a margin for the drift of the CG's
  recursive residual;
* the intracellular step at sampled occupied voxels that do not commit:
  the oracle's `ode_step` from the state before the step and the solved
  oxygen, P and V_c to 1e-10, phi bit for bit;
* the CA at every committed cell (Algorithm 1's cell update): the committed
  set from the oracle's cycle increment, each cell's kill decision from the
  oracle's Philox uniforms and kill probabilities at its voxel index within
  its replicate; a killed cell's voxel is empty after the step, every other
  committed cell stays with phi = 0; each new cell has phi, P, V_c = 0 and a
  committed, surviving cell among its 26 neighbours; the library's event
  counts equal these.

The surrogate's outputs at scale are covered by test_gpu_mlp.py (a tiled
lattice of 2.36 M voxels against the 32^3 result) and the bench's
error_matched_inputs.
"""
import numpy as np
import pytest

import bench
from oracle import ca as oca
from oracle import lattice as olat
from oracle import model as om
from oracle import ode as oode
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

RES_TOL = 2e-10     # CG stopping tolerance 1e-10, with a margin for recursion drift
ODE_TOL = 1e-10
NAMES = ("L", "K", "G1", "G2", "P", "Vc", "phi")


def moore():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dz, dy, dx) != (0, 0, 0)]


def test_headline_workload_step_against_the_oracle():
    reps, _, _ = bench.make_workload("config5")
    print(f"\n[full size] {len(reps)} x {reps[0][0].shape} voxels, default parameters", flush=True)
    with hca.Simulation(reps, hca.default_params()) as sim:
        sim.step(2)
        old = [{k: sim.field(k, r) for k in NAMES} for r in range(len(reps))]
        steps = [sim.stats(r)["step"] for r in range(len(reps))]
        sim.step()
        new = [{k: sim.field(k, r) for k in NAMES} for r in range(len(reps))]
        stats = [sim.stats(r) for r in range(len(reps))]
    rng = np.random.default_rng(7)
    for r, (cell, w, seed, (times, amts)) in enumerate(reps):
        o, n, st, step = old[r], new[r], stats[r], steps[r]
        assert step == 2 and st["step"] == 3, (step, st["step"])
        sched = om.Schedule(times=times, amts=amts)
        # the solves: true residual of the library's fields in the oracle's systems
        g0 = om.plasma_pair((step + 1) * OP.dt_min, sched, OP)
        systems = (("K", om.o2_system(o["L"], w, o["K"], OP), OP.a_K),
                   ("G1", om.drug_system(w, o["G1"], g0[0], OP), OP.a_G),
                   ("G2", om.drug_system(w, o["G2"], g0[1], OP), OP.a_G))
        for name, (c, b), a in systems:
            res = b - olat.operator_apply(c, a, n[name])
            rel = np.linalg.norm(res) / np.linalg.norm(b)
            print(f"[full size] replicate {r} {name}: true rel. residual {rel:.2e}", flush=True)
            assert rel <= RES_TOL, (r, name, rel)
        # the cells that commit this step, from the oracle's cycle increment
        K = np.maximum(n["K"], 0.0)
        can = o["L"] == 1
        phi_ode = o["phi"].copy()
        phi_ode[can] = o["phi"][can] + oode.cycle_increment(K[can], OP.dt_min, OP)
        committed = can & (phi_ode >= 1.0)
        # the intracellular step at sampled occupied voxels that do not commit
        pool = np.flatnonzero((o["L"] != 0) & ~committed)
        idx = rng.choice(pool, size=min(4096, pool.size), replace=False)
        P_s, V_s, f_s = oode.ode_step(o["L"].ravel()[idx], n["K"].ravel()[idx], o["P"].ravel()[idx],
                                      o["Vc"].ravel()[idx], o["phi"].ravel()[idx], OP)
        for name, ref in (("P", P_s), ("Vc", V_s)):
            got = n[name].ravel()[idx]
            assert np.abs(got - ref).max() <= ODE_TOL * np.abs(ref).max(), (r, name)
        assert np.array_equal(n["phi"].ravel()[idx], f_s), r
        assert np.array_equal(n["L"].ravel()[idx], o["L"].ravel()[idx]), r
        # the CA at every committed cell: kill trials at the cells' voxel indices
        gids = np.flatnonzero(committed)
        u0, u1, _ = oca.kill_uniforms(gids, step, seed)
        p1 = oca.kill_probability(n["G1"].ravel()[gids], OP.G_ref[0], OP.b_int[0])
        p2 = oca.kill_probability(n["G2"].ravel()[gids], OP.G_ref[1], OP.b_int[1])
        killed = (u0 < p1) | (u1 < p2)
        Ln = n["L"].ravel()
        print(f"[full size] replicate {r}: {gids.size} committed, {killed.sum()} killed", flush=True)
        assert gids.size > 0 and killed.any() and not killed.all(), r
        assert np.all(Ln[gids[killed]] == 0), r
        assert np.all(Ln[gids[~killed]] == 1), r
        assert np.all(n["phi"].ravel()[gids] == 0.0), r
        for name in ("P", "Vc"):
            assert np.all(n[name].ravel()[gids[killed]] == 0.0), (r, name)
        # new cells: reset state and a committed, surviving parent among the neighbours
        born = np.flatnonzero((o["L"].ravel() == 0) & (Ln == 1))
        for name in ("phi", "P", "Vc"):
            assert np.all(n[name].ravel()[born] == 0.0), (r, name)
        parent = np.zeros(committed.size, dtype=bool)
        parent[gids[~killed]] = True
        nz, ny, nx = cell.shape
        bz, rem = np.divmod(born, ny * nx)
        by, bx = np.divmod(rem, nx)
        has_parent = np.zeros(born.size, dtype=bool)
        for dz, dy, dx in moore():
            z, y, x = bz + dz, by + dy, bx + dx
            ok = (z >= 0) & (z < nz) & (y >= 0) & (y < ny) & (x >= 0) & (x < nx)
            j = (np.clip(z, 0, nz - 1) * ny + np.clip(y, 0, ny - 1)) * nx + np.clip(x, 0, nx - 1)
            has_parent |= ok & parent[j]
        assert has_parent.all(), r
        # the library's counts of this step
        assert st["committed"] == gids.size, r
        assert st["kills"] == killed.sum(), r
        assert st["divisions"] == born.size, r
        assert (Ln == 1).sum() == can.sum() - killed.sum() + born.size, r
