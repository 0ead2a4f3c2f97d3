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
of the timed steps (inputs resident in HBM, init excluded).  ``roofline`` is
the dominant kernel's algorithmic bytes per launch / its mean launch time from
HIP events recorded on the library's stream during the timed steps.
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample on one core.
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(budget_s=20.0):
    """The oracle as it stands (sparse-LU solves, NumPy ODE/CA) on one core,
    timed on whole coupled steps of the 32^3 lattice of the same recipe."""
    from threadpoolctl import threadpool_limits

    from oracle import model as om
    from oracle.constants import DEFAULT as OP
    from paper_2105_00448_amd import synth
    tis = synth.make_tissue(32, 8, seed=1)
    sched = synth.bolus_schedule([0, 50])
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    with threadpool_limits(limits=1):
        s = om.init_state(tis.cell, tis.w, tis.seed, OP)
        t0 = time.perf_counter()
        n = 0
        while True:
            s, _ = om.step(s, tis.w, osched, tis.seed, OP)
            n += 1
            el = time.perf_counter() - t0
            if el > budget_s or n >= 50:
                break
    vox = tis.cell.size
    return {"value": vox * n / el, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} coupled steps of a 32^3 lattice (same generator recipe), FP64 "
                      f"sparse-LU solves, single thread, {el:.1f}s; host: {cpu_model()}, "
                      f"{os.cpu_count()} logical CPUs"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicates and z-slabs would shard across GPUs; see the design notes).",
              file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_2105_00448_amd import hca
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    print(f"[bench] generating workload {args.workload}", file=sys.stderr, flush=True)
    reps, cfg, cfg_steps = make_workload(args.workload)
    solver_kw = {"precond": args.precond}
    if args.mg_coarse_max is not None:
        solver_kw["mg_coarse_max"] = args.mg_coarse_max
    steps = args.steps if args.steps is not None else cfg_steps
    nvox = sum(r[0].size for r in reps)

    # warm-up on a throwaway context (code loading, clocks), then the timed
    # run from step 0 of the workload
    if args.warmup > 0:
        p = hca.default_params(**solver_kw)
        with hca.Simulation(reps, p, stream=stream) as sim:
            sim.step(args.warmup)
        print(f"[bench] warm-up {args.warmup} steps done", file=sys.stderr, flush=True)

    p = hca.default_params(profile=0 if args.no_profile else 1, **solver_kw)
    t_init = time.perf_counter()
    sim = hca.Simulation(reps, p, stream=stream)
    t_init = time.perf_counter() - t_init
    print(f"[bench] init {t_init:.2f}s, timing {steps} steps", file=sys.stderr, flush=True)
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
    sim.close()
    print(f"[bench] {steps} steps in {el:.3f}s", file=sys.stderr, flush=True)

    value = nvox * steps / el
    rec = {
        "metric": "voxel-steps/s per GPU (plain coupled step)",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, precond="jacobi" if args.precond == 0 else "multigrid",
                       mg_coarse_max=p.mg_coarse_max),
    }
    if not args.no_profile:
        real = {k: v for k, v in kt.items() if v["launches"] > 0 and v["bytes_per_launch"] > 0}
        dom = max(real, key=lambda k: real[k]["ms"])
        d = real[dom]
        mean_s = d["ms"] / d["launches"] * 1e-3
        achieved = d["bytes_per_launch"] / mean_s / 1e9
        rec["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": None, "mean_launch_us": mean_s * 1e6,
                           "launches": d["launches"],
                           "bytes_per_launch": d["bytes_per_launch"]}
        tot = sum(v["ms"] for v in kt.values())
        rec["kernel_share"] = {k: round(v["ms"] / tot, 4) for k, v in kt.items() if v["ms"] > 0}
    rec["solver"] = {"cg_iters_last_step": st[0]["cg_iters"],
                     "relres_last_step": st[0]["cg_relres"]}
    rec["cells"] = {"cancer": sum(s["n_cancer"] for s in st),
                    "divisions": sum(s["total_divisions"] for s in st),
                    "kills": sum(s["total_kills"] for s in st)}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
