"""Benchmark of the coupled HCA time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config5] [--legs ...]

Headline (default ``--workload config5``), the metric "voxel-steps/s per GPU:
plain vs surrogate+batched at matched error/flip rate" on its largest
single-GPU configuration: 4 replicates (seeds 5000..5003) of a 384^3 lattice
(56.6M voxels each, 226M in one context), density from 512 Gaussians, 10 %
lognormal vessels, both drugs dosed at steps 0 and 100, 200 coupled steps of
30 min (K of them timed with --steps), FP64 fields.  The ODE surrogate is
trained first on the GPU (10^6 pairs harvested from the plain integrator on
32^3 lattices, 4000 Adam steps); then two contexts of the same lattices, each
init + W warm-up steps + K timed steps (inputs resident, no events, CG
iterations replayed from HIP graphs), then a few event-timed steps of the same
context for the kernel shares, the roofline kernel and the MFMA kernel:
  ``plain``   the plain intracellular integrator;
  ``value``   surrogate ODE (fallback within 1e-3 of phi = 1) + batched.
Also: the per-step error and decision-flip rate of the surrogate against the
plain integrator on identical inputs (replicate 0, 3 steps), the whole step's
algorithmic HBM bytes per voxel-step and their rate, the MFMA utilisation of
the surrogate kernel, and the paper's own CPU-cluster figures as context.
``cpu_baseline`` times the FP64 CPU oracle on one core on a 32^3 block of the
headline workload's first replicate.

Legs (``--legs``, comma-separated; default plain128,batched):
  plain128   the 128^3 plain workload (64 Gaussians, boluses at steps 0 and
             50), median of 3 runs from fresh contexts, with its roofline;
  batched    64 replicates of cubic edge U{48..96}, per-replicate seed and
             schedule, 50 steps, autotuned tiles;
  fp32       the headline lattices plain and surrogate with the solved fields
             stored in FP32 (precision 32);
  cpu_wide   the oracle on the 128^3 workload's first 5 steps (extrapolated)
             and on 4 ensemble replicates in 4 processes (minutes);
  surrogate  the 256^3 surrogate workload; substeps, newton, paper2d, vegf,
             fec: the options of the model on the 128^3 workload (see the
             leg functions).

``--profile-only`` (for rocprofv3 runs): one context of the workload stepped
W + K times, nothing else timed.
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
    if name == "config5":
        reps = []
        sched = synth.bolus_schedule([0, 100])
        for r in range(4):
            tis = synth.make_tissue(384, 512, seed=5000 + r)
            reps.append((tis.cell, tis.w, tis.seed, (sched.times, sched.amts)))
        cfg = {"workload": "largest single-GPU domain: 4 replicates (Philox seeds 5000..5003) of a "
                           "384^3 lattice (h=20um, 56.6M voxels each, 226M in one context), "
                           "heterogeneous density from 512 Gaussians, 10% lognormal vessels, O2 + 2 "
                           "drugs (bolus of both at steps 0 and 100), implicit Euler dt=30min, FP64 "
                           "MG-CG to rel. res. 1e-10; surrogate ODE (MLP 6-64-64-64-3, BF16 MFMA) with "
                           "plain-integrator fallback within 1e-3 of phi = 1; all replicates batched "
                           "in one launch per phase",
               "lattice": [384, 384, 384], "replicates": 4, "seeds": [5000, 5001, 5002, 5003],
               "gaussians": 512, "config_steps": 200}
        return reps, cfg, 200
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


def measured_traffic(kernel, workload, bytes_per_launch=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size): its
    measured bytes per voxel times this launch's active voxels (algorithmic
    bytes per launch / algorithmic bytes per voxel); None if the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    if "traffic_bytes_per_voxel" in rec and bytes_per_launch:
        return rec["traffic_bytes_per_voxel"] / rec["algorithmic_bytes_per_voxel"] * bytes_per_launch
    return rec.get("traffic_bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(crop=None, budget_s=12.0):
    """The oracle as it stands (CG solves to rel. residual 1e-15, NumPy ODE and
    CA) on one core, repeated until about `budget_s` seconds of stepping:
    20 coupled steps from init of `crop` = (cell, w, seed, (times, amts)), a
    32^3 block of the headline workload's first replicate (same generator,
    its dose schedule; zero-flux faces at the block's edges), or of the 32^3
    8-Gaussian workload (seed 1, bolus at step 0) without one."""
    from threadpoolctl import threadpool_limits

    from oracle import model as om
    from oracle.constants import DEFAULT as OP
    from paper_2105_00448_amd import synth
    if crop is None:
        tis = synth.make_tissue(32, 8, seed=1)
        sched = synth.bolus_schedule([0])
        cell, w, seed, (times, amts) = tis.cell, tis.w, tis.seed, (sched.times, sched.amts)
        what = "the 32^3 workload (8-Gaussian density, seed 1, bolus at step 0) in full"
    else:
        cell, w, seed, (times, amts) = crop
        what = ("a 32^3 block (voxels [0,32)^3) of the headline workload's first 384^3 replicate "
                f"(512-Gaussian density, seed {seed}, its bolus at step 0)")
    osched = om.Schedule(times=times, amts=amts)
    el, n, runs = 0.0, 0, 0
    with threadpool_limits(limits=1):
        while el < budget_s:
            s = om.init_state(cell, w, seed, OP)
            t0 = time.perf_counter()
            for _ in range(20):
                s, _ = om.step(s, w, osched, seed, OP)
            el += time.perf_counter() - t0
            n += 20
            runs += 1
    vox = cell.size
    return {"value": vox * n / el, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}, 20 coupled steps from init, {runs} runs ({n} steps, {el:.1f}s of "
                      f"stepping, init excluded); FP64 diagonally scaled CG to rel. residual 1e-15, "
                      f"single thread; host: {cpu_model()}, {os.cpu_count()} logical CPUs"}


def _oracle_steps(args):
    """Worker of cpu_wide: (cell, w, seed, times, amts, steps) -> (voxels, steps, seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import model as om
    from oracle.constants import DEFAULT as OP
    cell, w, seed, times, amts, steps = args
    with threadpool_limits(limits=1):
        s = om.init_state(cell, w, seed, OP)
        sched = om.Schedule(times=times, amts=amts)
        t0 = time.perf_counter()
        for _ in range(steps):
            s, _ = om.step(s, w, sched, seed, OP)
        return cell.size, steps, time.perf_counter() - t0


def cpu_wide():
    """The oracle on the larger workloads (minutes of CPU time; off by
    default): the 128^3 workload over its first 5 steps (its 100-step run
    extrapolated from them, labelled so), and 4 replicates of the
    64-replicate ensemble, one process each."""
    import multiprocessing as mp
    reps, _, _ = make_workload("plain128")
    cell, w, seed, (times, amts) = reps[0]
    print("[bench:cpu_wide] oracle, 128^3, 5 steps", file=sys.stderr, flush=True)
    nv, ns, el = _oracle_steps((cell, w, seed, times, amts, 5))
    out = {"plain128_first5": {"value": nv * ns / el, "unit": "voxel-steps/s", "cores": 1,
                               "seconds_5_steps": el,
                               "extrapolated_100_steps_s": el * 20,
                               "note": "5 steps after init, extrapolated linearly to 100"}}
    ens, _, _ = make_workload("batched64")
    jobs = [(c, ww, sd, tm, am, 50) for c, ww, sd, (tm, am) in ens[:4]]
    print("[bench:cpu_wide] oracle, 4 ensemble replicates x 50 steps, 4 processes",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(4) as pool:
        res = pool.map(_oracle_steps, jobs)
    wall = time.perf_counter() - t0
    vs = sum(r[0] * r[1] for r in res)
    out["batched4"] = {"value": vs / max(r[2] for r in res), "unit": "voxel-steps/s", "cores": 4,
                       "replicates": [list(c.shape) for c, *_ in jobs], "steps": 50,
                       "wall_s_incl_init": wall,
                       "note": "4 of the 64 replicates, one process each; value from the slowest "
                               "process's stepping time (init excluded)"}
    out["host"] = f"{cpu_model()}, {os.cpu_count()} logical CPUs"
    return out


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


# MI355X dense bf16 MFMA peak (no sparsity), FLOP/s
MFMA_BF16_PEAK = 2.5e15
# network flops per voxel: algorithmic (2 x multiply-adds of 6-64-64-64-3) and as
# executed on 32x32x16 tiles (6 inputs padded to 16, 3 outputs to 32)
MLP_FLOP_ALG = 2 * (6 * 64 + 64 * 64 + 64 * 64 + 64 * 3)
MLP_FLOP_EXEC = 2 * (64 * 16 + 64 * 64 + 64 * 64 + 32 * 64)
# the paper's own CPU figures for this path (its weak-scaling tables), context only
PAPER_CONTEXT = {
    "hardware": "Saga (NTNU): Intel Xeon Gold 6138 @ 2.0 GHz, 40 cores and 192 GiB per node, "
                "1 to 80 cores; FEniCS 2019.1.0 + PETSc + hypre BoomerAMG",
    "discretisation": "2-D P1 finite elements on a 4x refined mesh (~16 dofs per lattice node), "
                      "Crank-Nicolson, 30 x 1-min PDE steps per 30-min update; not like-for-like",
    "chemo_update_1core": {"dofs": 159197, "assembly_s": 2.9177, "solve_s": 6.2043},
    "chemo_update_80cores": {"dofs": 12809237, "assembly_s": 3.7708, "solve_s": 15.784},
    "o2_linearised_update_1core": {"assembly_s": 2.6657, "solve_s": 3.0532},
    "o2_linearised_update_80cores": {"assembly_s": 3.5985, "solve_s": 6.8429},
    "derived_dof_steps_per_s_1core_o2": 8.4e5,
    "derived_dof_steps_per_s_80cores_o2": 3.7e7,
}


def train_surrogate(stream, train_steps, n_pairs=1_000_000):
    """Training pairs harvested from the plain integrator on 32^3 lattices
    (seeds 1..6, 20 steps each, truncated to n_pairs), the network trained
    on the GPU by the library's kernels; returns (trainer, net, info)."""
    import torch

    from paper_2105_00448_amd import hca, synth
    dev = torch.device("cuda", 0)
    log = lambda m: print(f"[bench:train] {m}", file=sys.stderr, flush=True)
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
    flop_per_sample = 3 * MLP_FLOP_ALG   # forward + two backward products
    info = {"pairs": int(X.shape[0]), "harvest_s": t_harvest, "steps": train_steps,
            "batch": batch, "seconds": t_train, "samples_per_s": train_steps * batch / t_train,
            "tflops": train_steps * batch * flop_per_sample / t_train / 1e12,
            "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-50:].mean())}
    # throughput against the batch (workgroups per step = batch / 64), on a
    # second trainer so that the network above is untouched
    sweep = []
    tr2 = hca.Trainer(X, Y, seed=2, stream=stream)
    for b in (4096, 16384, 65536):
        n = 50
        tr2.train(2, batch=b, lr=1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr2.train(n, batch=b, lr=1e-4)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sweep.append({"batch": b, "workgroups": b // 64, "us_per_step": dt / n * 1e6,
                      "samples_per_s": n * b / dt, "tflops": n * b * flop_per_sample / dt / 1e12})
    tr2.close()
    info["batch_sweep"] = sweep
    return tr, tr.export(), info


def kernel_window(sim, names, steps, profile):
    """`steps` further coupled steps of a live context with params.profile =
    `profile`; returns the kernel table of that window."""
    sim.set_profile(profile)
    sim.reset_kernel_times()
    sim.step(steps)
    kt = sim.kernel_times()
    sim.set_profile(0)
    return kt


def run_context(reps, params, warmup, steps, stream, net=None, margin=1e-3, prof_steps=3,
                label="", repeats=1, runner_up=True):
    """`repeats` times: init a fresh context, `warmup` untimed steps, `steps`
    timed steps (no events, graphs replayed); `el` is the median of the timed
    runs (`els` all of them).  Then two short profiled windows on the last
    context: every kernel class (time shares, algorithmic bytes of a step) and
    the dominant class alone (its launch durations); the runner-up class too
    when its time is within 15 % of the dominant one's (the two can trade
    places from window to window)."""
    import statistics

    import torch

    from paper_2105_00448_amd import hca
    names = [hca.lib().hca_kernel_name(k).decode() for k in range(hca.lib().hca_num_kernels())]
    els = []
    sim = None
    for rep_i in range(repeats):
        if sim is not None:
            sim.close()
            torch.cuda.empty_cache()
        t0 = time.perf_counter()
        sim = hca.Simulation(reps, params, stream=stream)
        t_init = time.perf_counter() - t0
        if net is not None:
            sim.set_surrogate(net, margin)
        print(f"[bench:{label}] run {rep_i + 1}/{repeats}: init {t_init:.1f}s; {warmup} warm-up steps",
              file=sys.stderr, flush=True)
        sim.step(warmup)
        torch.cuda.synchronize()
        sim.synchronize()
        print(f"[bench:{label}] timing {steps} steps", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        torch.cuda.synchronize()
        els.append(time.perf_counter() - t0)
        print(f"[bench:{label}] {steps} steps in {els[-1]:.3f}s", file=sys.stderr, flush=True)
    el = statistics.median(els)
    st = [sim.stats(r) for r in range(len(reps))]
    if prof_steps == 0:
        return {"el": el, "els": els, "init_s": t_init, "stats": st, "sim": sim, "dom": None}
    print(f"[bench:{label}] profiling {prof_steps} + {prof_steps} steps", file=sys.stderr, flush=True)
    kt_all = kernel_window(sim, names, prof_steps, 1)
    real = {k: v for k, v in kt_all.items() if v["launches"] > 0 and v["bytes_per_launch"] > 0}
    ranked = sorted(real, key=lambda k: -real[k]["ms"])
    dom = ranked[0]
    kt_dom = kernel_window(sim, names, prof_steps, names.index(dom) + 2)
    second, kt_second = None, None
    if runner_up and len(ranked) > 1 and real[ranked[1]]["ms"] >= 0.85 * real[dom]["ms"]:
        second = ranked[1]
        kt_second = kernel_window(sim, names, prof_steps, names.index(second) + 2)[second]
    kt_mlp = None
    if net is not None:
        kt_mlp = kernel_window(sim, names, prof_steps, names.index("k_mlp_apply") + 2)["k_mlp_apply"]
    out = {"el": el, "els": els, "init_s": t_init, "stats": st, "kt_all": kt_all, "dom": dom,
           "kt_dom": kt_dom[dom], "second": second, "kt_second": kt_second, "kt_mlp": kt_mlp,
           "sim": sim}
    return out


def surrogate_error_matched(reps, net, stream, err_steps=3, margin=1e-3):
    """Per-step error and decision flips of the surrogate ODE phase against
    the plain integrator on identical inputs (the first replicate: the plain
    context's state copied into the surrogate context before each phase)."""
    import torch

    from paper_2105_00448_amd import hca
    dev = torch.device("cuda", 0)
    rep0 = reps[:1]
    nvox = rep0[0][0].size
    errs = []
    with hca.Simulation(rep0, hca.default_params(), stream=stream) as p, \
            hca.Simulation(rep0, hca.default_params(), stream=stream) as s:
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
                d = (a[m] - b[m]).abs()
                e[k] = (d.max() / b[m].abs().max()).item()
                e[k + "_rms"] = (d.pow(2).mean().sqrt() / b[m].pow(2).mean().sqrt()).item()
                if k == "phi":
                    e["flips"] = int(((a[can] >= 1.0) != (b[can] >= 1.0)).sum().item())
                    e["cancer"] = int(can.sum().item())
            e["fallbacks"] = s.stats()["sur_fallbacks"]
            e["occupied"] = int(occ.sum().item())
            errs.append(e)
            p.run_phases(hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
    return {
        "steps": err_steps, "replicate": 0,
        "P_max_rel": max(e["P"] for e in errs), "Vc_max_rel": max(e["Vc"] for e in errs),
        "phi_max_rel": max(e["phi"] for e in errs),
        "P_rms_rel": max(e["P_rms"] for e in errs), "Vc_rms_rel": max(e["Vc_rms"] for e in errs),
        "phi_rms_rel": max(e["phi_rms"] for e in errs),
        "flip_rate": sum(e["flips"] for e in errs) / max(1, sum(e["cancer"] for e in errs)),
        "flips": sum(e["flips"] for e in errs),
        "fallback_frac": sum(e["fallbacks"] for e in errs) / max(1, sum(e["occupied"] for e in errs)),
    }


def step_bytes(kt_all, steps):
    """Algorithmic HBM bytes per coupled step summed over every kernel class
    of a profiled window, and the kernel time per step."""
    b = sum(v["launches"] * v["bytes_per_launch"] for v in kt_all.values())
    ms = sum(v["ms"] for v in kt_all.values())
    return b / steps, ms / steps


def roofline_of(kt_dom, dom, workload, elem=8):
    """Roofline object of the dominant kernel from its event-timed launches."""
    mean_s = kt_dom["ms"] / kt_dom["launches"] * 1e-3
    achieved = kt_dom["bytes_per_launch"] / mean_s / 1e9
    kname = dom.replace("<L0>", "_L0").split("<")[0]
    r = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS,
         "traffic": measured_traffic(kname, workload, kt_dom["bytes_per_launch"]),
         "traffic_source": f"profiles/{kname}_{workload}_traffic.json",
         "mean_launch_us": mean_s * 1e6, "launches": kt_dom["launches"],
         "bytes_per_launch": kt_dom["bytes_per_launch"]}
    if kname == "k_cg_update":
        # the kernel moves 8 B per voxel more than the CG's compulsory 3 stored
        # values r, q read and r written (the multigrid's FP32 z read and r copy
        # written; x += alpha p is made by the next apply)
        r["frac_incl_fp32_copies"] = r["frac"] * (3 * elem + 8.0) / (3 * elem)
    return r


def stream_ceiling():
    """Device-to-device streaming rates of plain torch kernels on 3.2 GB FP64
    arrays (a copy: 1 read + 1 write; an add: 2 reads + 1 write): what a
    simple streaming kernel attains on this GPU, beside the 8 TB/s peak."""
    import torch
    n = 400_000_000
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 16 * n),
                             ("add", lambda: torch.add(a, b, out=c), 24 * n)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_gbs"] = nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return out


def config5_headline(args, stream):
    """The metric's configuration: plain vs surrogate+batched on 4 x 384^3."""
    import torch

    from paper_2105_00448_amd import hca
    print("[bench] generating workload config5 (4 x 384^3, 512 Gaussians)", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    reps, cfg, cfg_steps = make_workload("config5")
    print(f"[bench] generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    steps = args.steps if args.steps is not None else cfg_steps
    nvox = sum(r[0].size for r in reps)
    cell0, w0, seed0, sched0 = reps[0]
    crop = (np.ascontiguousarray(cell0[:32, :32, :32]), np.ascontiguousarray(w0[:32, :32, :32]),
            seed0, sched0)
    ceiling = stream_ceiling()
    print(f"[bench] streaming ceiling {ceiling}", file=sys.stderr, flush=True)
    tr, net, train_info = train_surrogate(stream, args.train_steps)
    kw = {"graphs": args.graphs}

    def summary(run, label, elem=8):
        st = run["stats"]
        kt = run["kt_all"]
        b_step, kms = step_bytes(kt, 3)
        ms = run["el"] / steps * 1e3
        tot = sum(v["ms"] for v in kt.values())
        out = {"value": nvox * steps / run["el"], "ms_per_step": ms, "repeats": len(run["els"]),
               "value_min_time": nvox * steps / min(run["els"]),
               "ms_per_step_runs": [round(e / steps * 1e3, 3) for e in run["els"]],
               "init_s": run["init_s"],
               "cg_iters_last_step": st[0]["cg_iters"],
               "roofline": roofline_of(run["kt_dom"], run["dom"],
                                       "config5" if elem == 8 else "config5_fp32", elem),
               "hbm_whole_step": {"bytes_per_voxel_step_algorithmic": b_step / nvox,
                                  "achieved_gbs": b_step / (ms * 1e-3) / 1e9,
                                  "frac": b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "kernel_ms_per_step_profiled": kms},
               "kernel_share": {k: round(v["ms"] / tot, 4) for k, v in kt.items() if v["ms"] > 0},
               "cells": {"cancer": sum(x["n_cancer"] for x in st),
                         "divisions": sum(x["total_divisions"] for x in st),
                         "kills": sum(x["total_kills"] for x in st)}}
        if run.get("second"):
            wl = "config5" if elem == 8 else "config5_fp32"
            out["roofline_runner_up"] = roofline_of(run["kt_second"], run["second"], wl, elem)
            out["roofline_runner_up"]["share_vs_dominant"] = kt[run["second"]]["ms"] / kt[run["dom"]]["ms"]
        ode = kt.get("k_ode", {})
        if ode.get("launches"):
            out["ode_phase_ms"] = ode["ms"] / ode["launches"]
        return out

    # fresh-context repeats (value = their median; value_min_time = the
    # fastest, the paper's convention), about 100 timed steps per context at most
    repeats = max(1, min(args.repeats, 100 // max(1, steps)))
    plain = run_context(reps, hca.default_params(**kw), args.warmup, steps, stream, label="plain",
                        repeats=repeats)
    plain_rec = summary(plain, "plain")
    plain["sim"].close()
    del plain
    torch.cuda.empty_cache()
    sur = run_context(reps, hca.default_params(**kw), args.warmup, steps, stream, net=net,
                      label="surrogate", repeats=repeats)
    sur_rec = summary(sur, "surrogate")
    st = sur["stats"]
    m = sur["kt_mlp"]
    mlp_s = m["ms"] / max(1, m["launches"]) * 1e-3
    net_vox = sum(x["sur_voxels"] for x in st)
    mfma = {"kernel": "k_mlp_apply", "mean_launch_us": mlp_s * 1e6,
            "network_voxels_per_launch": net_vox,
            "fallback_voxels_per_launch": sum(x["sur_fallbacks"] for x in st),
            "flop_per_voxel_algorithmic": MLP_FLOP_ALG, "flop_per_voxel_executed": MLP_FLOP_EXEC,
            "achieved_tflops": net_vox * MLP_FLOP_ALG / mlp_s / 1e12,
            "peak_tflops_bf16_dense": MFMA_BF16_PEAK / 1e12,
            "utilisation": net_vox * MLP_FLOP_ALG / mlp_s / MFMA_BF16_PEAK,
            "utilisation_executed": net_vox * MLP_FLOP_EXEC / mlp_s / MFMA_BF16_PEAK,
            "hbm_gbs": m["bytes_per_launch"] / mlp_s / 1e9,
            "ode_phase_ms_surrogate": mlp_s * 1e3,
            "ode_phase_ms_plain": plain_rec.get("ode_phase_ms")}
    sur["sim"].close()
    del sur
    torch.cuda.empty_cache()
    print("[bench] error at matched inputs, 3 steps on replicate 0", file=sys.stderr, flush=True)
    err = surrogate_error_matched(reps, net, stream)
    fp32 = None
    if "fp32" in args.legs.split(",") and not args.no_legs:
        # the same lattices with the solved fields stored in FP32 (solves to
        # relative residual 1e-8, the FP32 floor)
        fp32 = {"workload": "the headline lattices (4 x 384^3) with precision 32: solved fields and "
                            "solver arrays stored in FP32, FP64 arithmetic, solves to rel. res. 1e-8"}
        for label, use_net in (("plain", None), ("surrogate", net)):
            run = run_context(reps, hca.default_params(precision=32, **kw), args.warmup, steps,
                              stream, net=use_net, label=f"fp32-{label}")
            fp32[label] = summary(run, label, elem=4)
            run["sim"].close()
            del run
            torch.cuda.empty_cache()
        fp32["speedup_vs_fp64_plain"] = fp32["plain"]["value"] / plain_rec["value"]
        fp32["speedup_vs_fp64_surrogate"] = fp32["surrogate"]["value"] / sur_rec["value"]
    tr.close()
    rec = {
        "metric": "voxel-steps/s per GPU: plain vs surrogate+batched at matched error/flip rate",
        "value": sur_rec["value"],
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": sur_rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, mode="surrogate ODE + batched ensemble (4 replicates in one context)"),
        "roofline": dict(sur_rec["roofline"], stream_ceiling=ceiling,
                         frac_of_stream_copy=sur_rec["roofline"]["achieved"] / ceiling["copy_gbs"]),
        "repeats": sur_rec["repeats"],
        "value_min_time": sur_rec["value_min_time"],
        "ms_per_step_runs": sur_rec["ms_per_step_runs"],
        "plain": {k: plain_rec[k] for k in ("value", "ms_per_step", "repeats", "value_min_time",
                                             "ms_per_step_runs", "init_s", "cg_iters_last_step",
                                             "roofline", "roofline_runner_up", "hbm_whole_step",
                                             "ode_phase_ms")
                  if k in plain_rec},
        "speedup_vs_plain": sur_rec["value"] / plain_rec["value"],
        "error_matched_inputs": err,
        "hbm_whole_step": sur_rec["hbm_whole_step"],
        "mfma": mfma,
        "kernel_share": sur_rec["kernel_share"],
        "init_s": sur_rec["init_s"],
        "cells": sur_rec["cells"],
        "cells_plain": plain_rec["cells"],
        "training": train_info,
        "paper_context": PAPER_CONTEXT,
        "_cpu_sample": crop,
    }
    if "roofline_runner_up" in sur_rec:
        rec["roofline_runner_up"] = sur_rec["roofline_runner_up"]
    if fp32 is not None:
        rec["fp32"] = fp32
    return rec


def single_workload(args, stream, workload, repeats, config_steps=False):
    """One workload (plain128, batched64) stepped from fresh contexts: the
    median of `repeats` timed runs, the dominant kernel's roofline from one
    further event-timed run.  `config_steps`: the workload's own step count
    (a leg beside the headline), not --steps."""
    import torch

    from paper_2105_00448_amd import hca
    print(f"[bench] generating workload {workload}", file=sys.stderr, flush=True)
    reps, cfg, cfg_steps = make_workload(workload)
    solver_kw = {"precond": args.precond, "graphs": args.graphs, "autotune": args.autotune}
    if args.mg_coarse_max is not None:
        solver_kw["mg_coarse_max"] = args.mg_coarse_max
    steps = cfg_steps if config_steps or args.steps is None else args.steps
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
    for rep_i in range(repeats):
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
        kname = dom.replace("<L0>", "_L0").split("<")[0]
        wname = workload
        rec["profiled_repeat_ms_per_step"] = el_prof / steps * 1e3
        rec["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(kname, wname, d["bytes_per_launch"]),
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
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="config5", help="config5 (headline), plain128, batched64")
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
    ap.add_argument("--legs", default="plain128,batched",
                    help="comma-separated further legs: plain128, batched, surrogate, substeps, newton, "
                         "paper2d, vegf, fec, cpu_wide")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--profile-only", action="store_true",
                    help="for profiler runs: train the network, then init one context of the "
                         "workload (config5: surrogate + batched; --precision) and step it "
                         "--warmup + --steps times; prints a short JSON line")
    ap.add_argument("--precision", type=int, default=64, help="with --profile-only: 64 or 32")
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
    if args.profile_only:
        reps, cfg, cfg_steps = make_workload(args.workload)
        steps = args.steps if args.steps is not None else cfg_steps
        net = None
        if args.workload == "config5":
            tr, net, _ = train_surrogate(stream, args.train_steps)
        p = hca.default_params(precision=args.precision, graphs=args.graphs)
        # the headline's context and profiled windows (every class, then the
        # dominant class alone, then the surrogate's), so that a kernel trace
        # of this run covers the launches the headline's roofline times
        run = run_context(reps, p, args.warmup, steps, stream, net=net,
                          prof_steps=3 if args.workload == "config5" else 0, label="profile-only",
                          runner_up=False)
        nvox = sum(r[0].size for r in reps)
        out = {"workload": args.workload, "precision": args.precision, "steps": steps,
               "ms_per_step": run["el"] / steps * 1e3, "value": nvox * steps / run["el"],
               "dominant_kernel": run["dom"]}
        if run["dom"] is not None:
            out["dominant_mean_launch_us"] = run["kt_dom"]["ms"] / run["kt_dom"]["launches"] * 1e3
        print(json.dumps(out), flush=True)
        run["sim"].close()
        return
    if args.workload == "config5":
        rec = config5_headline(args, stream)
    else:
        rec = single_workload(args, stream, args.workload, args.repeats)
    legs = [] if args.no_legs else [x for x in args.legs.split(",") if x]
    crop = rec.pop("_cpu_sample", None)
    if "plain128" in legs and args.workload != "plain128":
        rec["plain128"] = single_workload(args, stream, "plain128", 3, config_steps=True)
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
        rec["cpu_baseline"] = cpu_baseline(crop)
    if "cpu_wide" in legs:
        rec["cpu_wide"] = cpu_wide()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
