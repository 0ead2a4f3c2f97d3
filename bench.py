"""Benchmark of the coupled HCA time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain128]

Workloads (all synthetic, seeded; generator recipe in paper_2105_00448_amd/synth.py):
  plain128   128^3 lattice, density from 64 Gaussians, 10% vessels, both drugs
             dosed at steps 0 and 50, 100 coupled steps of 30 min, FP64 fields,
             solves to relative residual 1e-10.   (default)
  batched64  64 replicates, cubic edges ~ U{48..96}, per-replicate seed and
             schedule (dose x U[0.5,1.5] on day {0,1,2}), 50 steps, one launch
             per phase kernel for the whole batch.

Prints ONE JSON line.  ``value`` is voxel-steps/s = voxels x steps / wall time
of the timed steps (inputs resident in HBM, init excluded), the median of
``--repeats`` timed runs from a fresh context each.  ``roofline`` is the
dominant kernel's algorithmic bytes per launch / its mean duration, from
start/stop events carried by that kernel's launches on the library's stream
during one further timed run of the same workload (events on every launch of
the other runs would slow them; that run's step time is reported as
``profiled_repeat_ms_per_step``).
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample on one core.

Two further legs (skip with --no-legs) report the other throughputs of the
same metric beside the plain one:
  surrogate  10^6 training pairs harvested from the plain integrator on 32^3
             lattices (seeds 1..6, 20 steps each), the network trained on the GPU,
             then the 256^3 lattice (64 Gaussians, bolus at steps 0 and 50)
             stepped plain and with the surrogate ODE phase (margin 1e-3), and
             the per-step error and decision-flip rate of the surrogate against
             the plain integrator on identical inputs;
  batched    the batched64 ensemble;
  substeps   the plain 128^3 workload with the paper's field time step: 30
             implicit 1-min substeps per 30-min coupled step, backward Euler
             and Crank-Nicolson (10 coupled steps each; off by default, add
             with --legs);
  newton     the plain 128^3 workload with 3 Newton steps on the nonlinear
             oxygen uptake after each linearised solve: step time, and the
             linearisation gap max|K_newton - K_linearised| / max K at matched
             inputs over 5 steps (off by default, add with --legs);
  paper2d    the paper's solver-performance setting as synthetic input: a 2-D
             1 mm^2 slice of 100 x 100 voxels of 10 um, cell and vascular
             densities 0.4 and 0.12, 30 Crank-Nicolson 1-min field substeps
             per 30-min update; one slice and a batch of 64 (off by default);
  vegf       the plain 128^3 workload with the extracellular VEGF field solved
             in the same batch as the other three and the vessel birth-death
             update every 720 min, 48 steps (two updates): step time beside
             the plain one, vessel events, and the vessel kernel's duration
             (off by default);
  fec        the plain 128^3 workload with the full FEC cocktail: epirubicin
             as a third drug (three-compartment plasma kinetics, its own
             tissue field and kill trial) dosed with the other two, 48 steps;
             alone, and with every option at once (exact Michaelis-Menten
             fluorouracil, VEGF and vessel updates: five fields per batched
             solve) (off by default).
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def make_workload(name):
    from paper_2105_00448_amd import synth
    if name == "plain128":
        tis = synth.make_tissue(128, 64, seed=2)
        sched = synth.bolus_schedule([0, 50])
        reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
        cfg = {"workload": "plain method at scale: 128^3 voxels (h=20um), 64-Gaussian density, "
                           "10% lognormal vessels, O2 + 2 drugs, bolus at steps 0 and 50, "
                           "implicit Euler dt=30min, FP64 CG to rel. res. 1e-10",
               "lattice": [128, 128, 128], "replicates": 1, "seed": 2, "config_steps": 100}
        return reps, cfg, 100
    if name == "batched64":
        ens = synth.ensemble(64, seed0=1000)
        reps = [(t.cell, t.w, t.seed, (s.times, s.amts)) for t, s in ens]
        edges = [t.cell.shape[0] for t, _ in ens]
        cfg = {"workload": "batched ensemble: 64 replicates, cubic edges U{48..96}, per-replicate "
                           "Philox seed and schedule (dose x U[0.5,1.5] on day 0/1/2), one launch "
                           "per phase kernel for the whole batch, FP64 CG to rel. res. 1e-10",
               "replicates": 64, "edges": edges, "config_steps": 50}
        return reps, cfg, 50
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or
    None if the kernel's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(budget_s=12.0):
    """The oracle as it stands (CG solves to rel. residual 1e-15, NumPy ODE and
    CA) on one core: the small workload in full (32^3 lattice, 8-Gaussian
    density, seed 1, bolus of both drugs at step 0, 20 coupled steps from
    init), repeated until about `budget_s` seconds of stepping."""
    from threadpoolctl import threadpool_limits

    from oracle import model as om
    from oracle.constants import DEFAULT as OP
    from paper_2105_00448_amd import synth
    tis = synth.make_tissue(32, 8, seed=1)
    sched = synth.bolus_schedule([0])
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    el, n, runs = 0.0, 0, 0
    with threadpool_limits(limits=1):
        while el < budget_s:
            s = om.init_state(tis.cell, tis.w, tis.seed, OP)
            t0 = time.perf_counter()
            for _ in range(20):
                s, _ = om.step(s, tis.w, osched, tis.seed, OP)
            el += time.perf_counter() - t0
            n += 20
            runs += 1
    vox = tis.cell.size
    return {"value": vox * n / el, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the 32^3 workload (8-Gaussian density, seed 1, bolus at step 0) in full, "
                      f"20 coupled steps from init, {runs} runs ({n} steps, {el:.1f}s of stepping, "
                      f"init excluded); FP64 diagonally scaled CG to rel. residual 1e-15, single "
                      f"thread; host: {cpu_model()}, {os.cpu_count()} logical CPUs"}


def timed_run(reps, params, steps, stream, net=None, margin=1e-3, tile_shapes=False):
    """Steps `steps` coupled steps of a fresh context; returns wall time,
    per-replicate stats and kernel times (and the tile shapes)."""
    import torch

    from paper_2105_00448_amd import hca
    sim = hca.Simulation(reps, params, stream=stream)
    if net is not None:
        sim.set_surrogate(net, margin)
    sim.reset_kernel_times()
    torch.cuda.synchronize()
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = [sim.stats(r) for r in range(len(reps))]
    kt = sim.kernel_times()
    shapes = [sim.tile_shape(r) for r in range(len(reps))]
    sim.close()
    if tile_shapes:
        return el, st, kt, shapes
    return el, st, kt


def surrogate_leg(stream, steps, train_steps, margin=1e-3, err_steps=3, edge=256,
                  n_pairs=1_000_000):
    import torch

    from paper_2105_00448_amd import hca, synth
    dev = torch.device("cuda", 0)
    log = lambda m: print(f"[bench:surrogate] {m}", file=sys.stderr, flush=True)
    # training pairs from the plain integrator
    t0 = time.perf_counter()
    Xs, Ys = [], []
    for seed in range(1, 7):
        tis = synth.make_tissue(32, 8, seed=seed)
        sched = synth.bolus_schedule([0])
        with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))],
                            hca.default_params(), stream=stream) as sim:
            X = torch.empty((tis.cell.size, 6), device=dev)
            Y = torch.empty((tis.cell.size, 3), device=dev)
            for _ in range(20):
                n = sim.harvest_step(X, Y)
                Xs.append(X[:n].clone())
                Ys.append(Y[:n].clone())
    X, Y = torch.cat(Xs)[:n_pairs].contiguous(), torch.cat(Ys)[:n_pairs].contiguous()
    del Xs, Ys
    t_harvest = time.perf_counter() - t0
    log(f"{X.shape[0]} pairs in {t_harvest:.1f}s; training {train_steps} steps")
    tr = hca.Trainer(X, Y, seed=1, stream=stream)
    batch = 4096
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l1 = tr.train(train_steps // 2, batch=batch, lr=2e-3)
    l2 = tr.train(train_steps - train_steps // 2, batch=batch, lr=5e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    losses = np.concatenate([l1, l2])
    flop_per_sample = 3 * 2 * (6 * 64 + 2 * 64 * 64 + 64 * 3)   # forward + two backward products
    net = tr.export()
    # the large lattice, plain and with the surrogate
    tis = synth.make_tissue(edge, 64, seed=4)
    sched = synth.bolus_schedule([0, 50])
    reps = [(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]
    nvox = tis.cell.size
    names = [hca.lib().hca_kernel_name(k).decode() for k in range(hca.lib().hca_num_kernels())]
    log(f"{edge}^3 plain, {steps} steps")
    el_p, st_p, kt_p = timed_run(reps, hca.default_params(profile=names.index("k_ode") + 2), steps,
                                 stream)
    log(f"{edge}^3 surrogate, {steps} steps")
    el_s, st_s, kt_s = timed_run(reps, hca.default_params(profile=names.index("k_mlp_apply") + 2),
                                 steps, stream, net, margin)
    ode_p = kt_p["k_ode"]["ms"] / max(1, kt_p["k_ode"]["launches"])
    ode_s = kt_s["k_mlp_apply"]["ms"] / max(1, kt_s["k_mlp_apply"]["launches"])
    # error and decision flips on identical inputs
    log(f"error at matched inputs, {err_steps} steps")
    errs = []
    with hca.Simulation(reps, hca.default_params(), stream=stream) as p, \
            hca.Simulation(reps, hca.default_params(), stream=stream) as s:
        s.set_surrogate(net, margin)
        buf8 = torch.empty(nvox, dtype=torch.float64, device=dev)
        buf1 = torch.empty(nvox, dtype=torch.uint8, device=dev)
        for _ in range(err_steps):
            p.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            for k in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
                b = buf1 if k == "L" else buf8
                p.field_to_device(k, b)
                s.set_field_from_device(k, b)
            p.run_phases(hca.PH_ODE)
            s.run_phases(hca.PH_ODE)
            L = p.field_to_device("L", torch.empty(nvox, dtype=torch.uint8, device=dev))
            occ, can = L != 0, L == 1
            e = {}
            for k in ("P", "Vc", "phi"):
                a = s.field_to_device(k, torch.empty(nvox, dtype=torch.float64, device=dev))
                b = p.field_to_device(k, torch.empty(nvox, dtype=torch.float64, device=dev))
                m = can if k == "phi" else occ
                e[k] = ((a[m] - b[m]).abs().max() / b[m].abs().max()).item()
                if k == "phi":
                    e["flips"] = int(((a[can] >= 1.0) != (b[can] >= 1.0)).sum().item())
                    e["cancer"] = int(can.sum().item())
            e["fallbacks"] = s.stats()["sur_fallbacks"]
            e["occupied"] = int(occ.sum().item())
            errs.append(e)
            p.run_phases(hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
    tr.close()
    return {
        "workload": f"surrogate ODE: {edge}^3 voxels, 64-Gaussian density, bolus at steps 0 and "
                    f"50, {steps} steps; network 6-64-64-64-3 GELU(erf), BF16 MFMA / FP32 "
                    f"accumulation; plain-integrator fallback within {margin} of phi = 1",
        "value_plain": nvox * steps / el_p,
        "value_surrogate": nvox * steps / el_s,
        "unit": "voxel-steps/s",
        "step_speedup": el_p / el_s,
        "ms_per_step_plain": el_p / steps * 1e3,
        "ms_per_step_surrogate": el_s / steps * 1e3,
        "ode_phase_ms_plain": ode_p,
        "ode_phase_ms_surrogate": ode_s,
        "ode_phase_speedup": ode_p / ode_s if ode_s > 0 else None,
        "fallback_frac_last_step": st_s[0]["sur_fallbacks"]
        / max(1, st_s[0]["sur_fallbacks"] + st_s[0]["sur_voxels"]),
        "n_cancer_end": {"plain": st_p[0]["n_cancer"], "surrogate": st_s[0]["n_cancer"]},
        "error_matched_inputs": {
            "steps": err_steps,
            "P_max_rel": max(e["P"] for e in errs),
            "Vc_max_rel": max(e["Vc"] for e in errs),
            "phi_max_rel": max(e["phi"] for e in errs),
            "flip_rate": sum(e["flips"] for e in errs) / max(1, sum(e["cancer"] for e in errs)),
            "fallback_frac": sum(e["fallbacks"] for e in errs) / max(1, sum(e["occupied"] for e in errs)),
        },
        "training": {"pairs": int(X.shape[0]), "harvest_s": t_harvest, "steps": train_steps,
                     "batch": batch, "seconds": t_train,
                     "samples_per_s": train_steps * batch / t_train,
                     "tflops": train_steps * batch * flop_per_sample / t_train / 1e12,
                     "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-50:].mean())},
    }


def batched_leg(stream, steps=None):
    from paper_2105_00448_amd import hca
    reps, cfg, cfg_steps = make_workload("batched64")
    steps = steps or cfg_steps
    nvox = sum(r[0].size for r in reps)
    print(f"[bench:batched] {len(reps)} replicates, {nvox} voxels, {steps} steps",
          file=sys.stderr, flush=True)
    el, st, _, shapes = timed_run(reps, hca.default_params(autotune=1), steps, stream,
                                  tile_shapes=True)
    dist = {}
    for t in shapes:
        k = "x".join(map(str, t))
        dist[k] = dist.get(k, 0) + 1
    return {"workload": cfg["workload"] + "; stencil tiles from the autotuner",
            "value": nvox * steps / el, "unit": "voxel-steps/s", "voxels": nvox, "steps": steps,
            "ms_per_step": el / steps * 1e3, "tile_shapes_txtytz": dist}


def substeps_leg(stream, steps=10, m=30):
    """The 128^3 workload with m field substeps per coupled step (backward
    Euler and Crank-Nicolson); value counts coupled steps, as the plain
    line does."""
    from paper_2105_00448_amd import hca
    reps, cfg, _ = make_workload("plain128")
    nvox = sum(r[0].size for r in reps)
    out = {"workload": f"plain 128^3 workload with {m} implicit field substeps of {30.0 / m:g} min per "
                       f"30-min coupled step, {steps} coupled steps",
           "unit": "voxel-steps/s"}
    for name, theta in (("backward_euler", 1.0), ("crank_nicolson", 0.5)):
        print(f"[bench:substeps] {name}, {m} substeps, {steps} steps", file=sys.stderr, flush=True)
        el, st, _ = timed_run(reps, hca.default_params(pde_substeps=m, pde_theta=theta), steps, stream)
        out[name] = {"value": nvox * steps / el, "ms_per_step": el / steps * 1e3,
                     "ms_per_substep": el / steps / m * 1e3,
                     "cg_iters_last_substep": list(st[0]["cg_iters"])}
    return out


def newton_leg(stream, steps=20, compare=5, newton=3):
    """The plain workload with `newton` Newton steps on the oxygen uptake:
    its step time beside the linearised one, and the gap between the two
    oxygen fields computed from the same state."""
    from paper_2105_00448_amd import hca
    reps, cfg, _ = make_workload("plain128")
    nvox = sum(r[0].size for r in reps)
    print(f"[bench:newton] {newton} Newton steps, {steps} steps", file=sys.stderr, flush=True)
    el_n, st_n, _ = timed_run(reps, hca.default_params(o2_newton=newton), steps, stream)
    el_l, _, _ = timed_run(reps, hca.default_params(), steps, stream)
    names = ("L", "K", "G1", "G2", "P", "Vc", "phi")

    def gaps_at_matched_inputs(m, n_steps):
        """(max-norm, 2-norm) relative gaps of K per step, m field substeps."""
        out = []
        kw = dict(pde_substeps=m)
        with hca.Simulation(reps, hca.default_params(**kw), stream=stream) as lin, \
                hca.Simulation(reps, hca.default_params(o2_newton=newton, **kw), stream=stream) as nwt:
            for k in range(n_steps):
                state = {n: lin.field(n) for n in names}
                lin.step(1)
                for n in names:
                    nwt.set_field(n, state[n])
                nwt.set_step(k)
                nwt.run_phases(hca.PH_O2 | hca.PH_DRUGS)
                Kl, Kn = lin.field("K"), nwt.field("K")
                out.append((float(np.abs(Kn - Kl).max() / np.abs(Kl).max()),
                            float(np.linalg.norm(Kn - Kl) / np.linalg.norm(Kl))))
        return out
    g30 = gaps_at_matched_inputs(1, compare)
    g1 = gaps_at_matched_inputs(30, 2)
    return {"workload": f"plain 128^3 workload, oxygen uptake at the new value by {newton} Newton steps "
                        f"after the linearised solve, {steps} steps",
            "unit": "voxel-steps/s", "value": nvox * steps / el_n,
            "ms_per_step": el_n / steps * 1e3, "ms_per_step_linearised": el_l / steps * 1e3,
            "cg_iters_last_step": list(st_n[0]["cg_iters"]),
            "linearisation_gap_30min_step": {"max_rel": max(g[0] for g in g30),
                                             "l2_rel": max(g[1] for g in g30), "per_step": g30},
            "linearisation_gap_1min_substeps": {"max_rel": max(g[0] for g in g1),
                                                "l2_rel": max(g[1] for g in g1), "per_step": g1},
            "paper_claim_gap": 3e-4}


def vegf_leg(stream, steps=48):
    """The plain workload with the VEGF option: step time and vessel events."""
    from paper_2105_00448_amd import hca
    reps, cfg, _ = make_workload("plain128")
    nvox = sum(r[0].size for r in reps)
    print(f"[bench:vegf] {steps} steps", file=sys.stderr, flush=True)
    el_v, st_v, _ = timed_run(reps, hca.default_params(vegf=1), steps, stream)
    el_p, _, _ = timed_run(reps, hca.default_params(), steps, stream)
    names = [hca.lib().hca_kernel_name(k).decode() for k in range(hca.lib().hca_num_kernels())]
    _, _, kt = timed_run(reps, hca.default_params(vegf=1, profile=1), steps, stream)
    ves = kt["k_vessel"]
    setup = kt["k_setup_step"]
    return {"workload": f"plain 128^3 workload with extracellular VEGF (4 fields per batched solve) and "
                        f"the vessel birth-death update every 720 min, {steps} steps",
            "unit": "voxel-steps/s", "value": nvox * steps / el_v,
            "ms_per_step": el_v / steps * 1e3, "ms_per_step_plain": el_p / steps * 1e3,
            "cg_iters_last_step": list(st_v[0]["cg_iters"]) + [st_v[0]["cg_iters_vegf"]],
            "vessel_births": st_v[0]["total_births"], "vessel_deaths": st_v[0]["total_deaths"],
            "n_vessel_end": st_v[0]["n_vessel"],
            "k_vessel_ms_per_launch": ves["ms"] / max(1, ves["launches"]),
            "k_vessel_launches": ves["launches"],
            "k_setup_step_ms_per_launch": setup["ms"] / max(1, setup["launches"]),
            "kernel_classes": len(names)}


def fec_leg(stream, steps=48):
    """The plain workload with the third drug, and with every option."""
    from paper_2105_00448_amd import hca
    reps, _, _ = make_workload("plain128")
    cell, w, seed, (times, amts) = reps[0]
    reps3 = [(cell, w, seed, (times + (times[0],), amts + (amts[0],)))]
    nvox = cell.size
    out = {"workload": f"plain 128^3 workload with epirubicin as a third drug dosed with the other two "
                       f"(steps 0 and 50), {steps} steps", "unit": "voxel-steps/s"}
    for name, kw in (("plain", {}), ("drug3", dict(drug3=1)),
                     ("all_options", dict(drug3=1, vegf=1, pk_mm=1))):
        print(f"[bench:fec] {name}, {steps} steps", file=sys.stderr, flush=True)
        el, st, _ = timed_run(reps3, hca.default_params(**kw), steps, stream)
        out[name] = {"value": nvox * steps / el, "ms_per_step": el / steps * 1e3,
                     "cg_iters_last_step": list(st[0]["cg_iters"]) + [st[0]["cg_iters_drug3"]],
                     "kills": st[0]["total_kills"], "cancer_end": st[0]["n_cancer"]}
    return out


def paper2d_leg(stream, steps=10, batch=64):
    """Time per 30-min update of the paper's 2-D performance setting."""
    from paper_2105_00448_amd import hca, synth
    prm = dict(h_um=10.0, pde_substeps=30, pde_theta=0.5)
    sched = synth.bolus_schedule([0])
    out = {"workload": "2-D slice 100 x 100 voxels of 10 um (1 mm^2), cell density 0.4, vascular density "
                       "0.12 (uniform, synthetic), bolus of both drugs at step 0, 30 Crank-Nicolson field "
                       f"substeps of 1 min per 30-min update, {steps} updates",
           "unit": "voxel-steps/s"}
    for n in (1, batch):
        tis = [synth.uniform_tissue((1, 100, 100), 0.4, 0.12, seed=500 + r) for r in range(n)]
        reps = [(t.cell, t.w, t.seed, (sched.times, sched.amts)) for t in tis]
        print(f"[bench:paper2d] {n} slice(s), {steps} updates", file=sys.stderr, flush=True)
        el, st, _ = timed_run(reps, hca.default_params(**prm), steps, stream)
        out[f"slices_{n}"] = {"value": n * 10000 * steps / el, "ms_per_update": el / steps * 1e3,
                              "cg_iters_last_substep": list(st[0]["cg_iters"])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain128")
    ap.add_argument("--precond", type=int, default=1, help="0 Jacobi, 1 multigrid")
    ap.add_argument("--mg-coarse-max", type=int, default=None,
                    help="levels with at most this many cells go to the one-workgroup solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--graphs", type=int, default=1, help="1: replay captured CG iterations")
    ap.add_argument("--autotune", type=int, default=0, help="1: tile plan from the autotuner")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats from a fresh context; value = median")
    ap.add_argument("--no-legs", action="store_true", help="plain workload only")
    ap.add_argument("--legs", default="surrogate,batched",
                    help="comma-separated further legs: surrogate, batched, substeps, newton, paper2d, "
                         "vegf, fec")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--sur-steps", type=int, default=100)
    ap.add_argument("--train-steps", type=int, default=4000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(replicates and z-slabs would shard across GPUs).",
              file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_2105_00448_amd import hca
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] copy calibration: 3 x {args.copy_calibration} MiB", file=sys.stderr,
              flush=True)
    print(f"[bench] generating workload {args.workload}", file=sys.stderr, flush=True)
    reps, cfg, cfg_steps = make_workload(args.workload)
    solver_kw = {"precond": args.precond, "graphs": args.graphs, "autotune": args.autotune}
    if args.mg_coarse_max is not None:
        solver_kw["mg_coarse_max"] = args.mg_coarse_max
    steps = args.steps if args.steps is not None else cfg_steps
    nvox = sum(r[0].size for r in reps)

    # warm-up on a throwaway context (code loading, clocks), every kernel
    # class timed to find the dominant one; then the timed run from step 0 of
    # the workload with HIP events around that class only (events around every
    # launch would add their own overhead to the timed steps)
    names = [hca.lib().hca_kernel_name(k).decode() for k in range(hca.lib().hca_num_kernels())]
    dom_class, warm_share = None, None
    if args.warmup > 0:
        p = hca.default_params(profile=0 if args.no_profile else 1, **solver_kw)
        with hca.Simulation(reps, p, stream=stream) as sim:
            sim.step(args.warmup)
            kt_w = sim.kernel_times()
        if not args.no_profile:
            real = {k: v for k, v in kt_w.items() if v["launches"] > 0 and v["bytes_per_launch"] > 0}
            dom_class = names.index(max(real, key=lambda k: real[k]["ms"]))
            tot = sum(v["ms"] for v in kt_w.values())
            warm_share = {k: round(v["ms"] / tot, 4) for k, v in kt_w.items() if v["ms"] > 0}
        print(f"[bench] warm-up {args.warmup} steps done", file=sys.stderr, flush=True)
    if dom_class is None and not args.no_profile:
        dom_class = names.index("k_cg_apply")

    # the timed repeats run as in production (no events, graphs replayed);
    # one further timed repeat carries HIP events around the dominant kernel
    # class only, for the roofline (events disable the graphs and add ~10 us
    # per event pair, so that repeat's step time is reported separately)
    def timed_repeat(prof, label):
        p = hca.default_params(profile=prof, **solver_kw)
        t_init = time.perf_counter()
        sim = hca.Simulation(reps, p, stream=stream)
        t_init = time.perf_counter() - t_init
        print(f"[bench] {label}: init {t_init:.2f}s, timing {steps} steps", file=sys.stderr,
              flush=True)
        sim.reset_kernel_times()
        torch.cuda.synchronize()
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        torch.cuda.synchronize()
        el_ = time.perf_counter() - t0
        st_ = [sim.stats(r) for r in range(len(reps))]
        kt_ = sim.kernel_times()
        mg_max = p.mg_coarse_max
        sim.close()
        print(f"[bench] {steps} steps in {el_:.3f}s", file=sys.stderr, flush=True)
        return el_, st_, kt_, mg_max

    times = []
    for rep_i in range(args.repeats):
        el1, st, _, mg_coarse_max = timed_repeat(0, f"repeat {rep_i}")
        times.append(el1)
    kt, el_prof = None, None
    if not args.no_profile:
        el_prof, _, kt, _ = timed_repeat(dom_class + 2, "profiled repeat")
    el = float(np.median(times))

    value = nvox * steps / el
    rec = {
        "metric": "voxel-steps/s per GPU (plain coupled step)",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3,
        "repeats": len(times),
        "value_min_time": nvox * steps / min(times),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, precond="jacobi" if args.precond == 0 else "multigrid",
                       mg_coarse_max=mg_coarse_max),
    }
    if not args.no_profile:
        dom = names[dom_class]
        d = kt[dom]
        mean_s = d["ms"] / d["launches"] * 1e-3
        achieved = d["bytes_per_launch"] / mean_s / 1e9
        kname = dom.split("<")[0]
        wname = args.workload
        rec["profiled_repeat_ms_per_step"] = el_prof / steps * 1e3
        rec["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(kname, wname),
                           "traffic_source": f"profiles/{kname}_{wname}_traffic.json",
                           "mean_launch_us": mean_s * 1e6,
                           "launches": d["launches"],
                           "bytes_per_launch": d["bytes_per_launch"]}
        if warm_share:
            rec["kernel_share_warmup"] = warm_share
    rec["solver"] = {"cg_iters_last_step": st[0]["cg_iters"],
                     "relres_last_step": st[0]["cg_relres"]}
    rec["cells"] = {"cancer": sum(s["n_cancer"] for s in st),
                    "divisions": sum(s["total_divisions"] for s in st),
                    "kills": sum(s["total_kills"] for s in st)}
    legs = [] if args.no_legs else [x for x in args.legs.split(",") if x]
    if "surrogate" in legs:
        rec["surrogate"] = surrogate_leg(stream, args.sur_steps, args.train_steps)
    if "batched" in legs:
        rec["batched"] = batched_leg(stream)
    if "substeps" in legs:
        rec["substeps"] = substeps_leg(stream)
    if "newton" in legs:
        rec["newton"] = newton_leg(stream)
    if "vegf" in legs:
        rec["vegf"] = vegf_leg(stream)
    if "fec" in legs:
        rec["fec"] = fec_leg(stream)
    if "paper2d" in legs:
        rec["paper2d"] = paper2d_leg(stream)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
