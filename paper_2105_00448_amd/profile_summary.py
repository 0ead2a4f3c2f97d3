"""Summaries of rocprofv3 runs of a bench workload, written under profiles/.

Reads three rocprofv3 output folders of the same `bench.py --profile-only`
command (a kernel trace, a FETCH_SIZE pass and a WRITE_SIZE pass, each
started with `--copy-calibration 256` so that the runtime's copy of 256 MiB
calibrates the counters) and writes:

  <workload>_kernel_stats.md              per-kernel durations of the stepped context
  <kernel>_<workload>_traffic.{json,md}   HBM bytes per voxel of the solver's
                                          streaming kernels (CG and level-0
                                          multigrid), against their algorithmic bytes

Usage: python -m paper_2105_00448_amd.profile_summary WORKLOAD PRECISION KT_DIR FETCH_DIR WRITE_DIR COMMAND
"""
import collections
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["paper_2105_00448_amd/csrc/k_solver.hip", "paper_2105_00448_amd/csrc/k_mg.hip",
           "paper_2105_00448_amd/csrc/dev_util.h", "paper_2105_00448_amd/csrc/hca_internal.h"]
COPY_KIB = 256 * 1024
# the counter passes collect only these dispatches (--kernel-include-regex)
PMC_REGEX = ("k_cg_update|k_cg_apply|k_cg_finish|k_mg_pre|k_mg_sweep|k_mg_restrict|k_mg_post1|k_mg_post2|"
             "k_mg_postfused|k_mg_coarse|k_init_cells|copyBuffer")
# kernels priced per launch (levels below level 0, the one-workgroup coarse solve)
PER_LAUNCH = ["k_mg_prefused<2>", "k_mg_postfused<2, false, double, double>",
              "k_mg_postfused<2, false, float, float>", "k_mg_pre<false, float>",
              "k_mg_restrict<false, float>", "k_mg_post1<false, float>",
              "k_mg_post2<false, float, double>", "k_mg_post2<false, float, float>", "k_mg_coarse"]
# voxels (of one system) of each workload, and its systems per solve
WORKLOADS = {"config5": (384 ** 3, 4), "plain128": (128 ** 3, 1)}


def kernels(e):
    """Streaming kernels of the solve (demangled-name prefix -> (short name,
    algorithmic bytes per active voxel)); e = bytes of a stored field value.
    Level 0 of the multigrid is the <true, ...> instance, or the fused
    three-stage passes k_mg_prefused<3> / k_mg_postfused<3, ...> (the default)."""
    fp = "double" if e == 8 else "float"
    return {
        f"k_cg_update<false, {fp}>": ("k_cg_update", 3 * e),
        f"k_cg_apply<false, {fp}>": ("k_cg_apply", 4 + 6 * e),
        f"k_cg_finish<{fp}>": ("k_cg_finish", 3 * e),
        "k_mg_pre<true, float>": ("k_mg_pre_L0", 12.0),
        "k_mg_sweep<true, float>": ("k_mg_sweep_L0", 16.0),
        "k_mg_restrict<true, float>": ("k_mg_restrict_L0", 12.5),
        "k_mg_post1<true, float>": ("k_mg_post1_L0", 16.5),
        f"k_mg_post2<true, {fp}, {fp}>": ("k_mg_post2_L0", 12 + e),
        "k_mg_prefused<3>": ("k_mg_prefused_L0", 12.5),
        f"k_mg_postfused<3, true, {fp}, {fp}>": ("k_mg_postfused_L0", 16.5 + e),
    }


def name(r):
    return r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hca::", "")


def one_csv(folder, suffix):
    hits = glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)
    if len(hits) != 1:
        raise SystemExit(f"expected one *{suffix} under {folder}, found {hits}")
    return list(csv.DictReader(open(hits[0])))


def stepped_context(rows, key):
    """Dispatches after the last context initialisation (k_init_cells)."""
    rows = sorted(rows, key=lambda r: int(r[key]))
    last = max(i for i, r in enumerate(rows) if "k_init_cells" in r["Kernel_Name"])
    return rows, rows[last + 1:]


def pmc_command(command, counter):
    """The counter pass of the kernel-trace command `command`."""
    return (command.replace("--kernel-trace --stats",
                            f"--pmc {counter} --kernel-include-regex '{PMC_REGEX}'")
            .replace("P_kt", "P_f" if counter == "FETCH_SIZE" else "P_w"))


def main(workload, precision, kt_dir, f_dir, w_dir, command):
    e = 8 if int(precision) == 64 else 4
    ks = kernels(e)
    nvox, nrep = WORKLOADS[workload]
    tag = workload if e == 8 else f"{workload}_fp32"
    _, kt = stepped_context(one_csv(kt_dir, "kernel_trace.csv"), "Start_Timestamp")
    dur = collections.defaultdict(list)
    for r in kt:
        dur[name(r)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in dur.values())
    span = (int(kt[-1]["End_Timestamp"]) - int(kt[0]["Start_Timestamp"])) / 1e6
    out = [f"# Kernel statistics: {tag} (multigrid-preconditioned CG, precision {precision})", "",
           "Command (repository root, one MI355X):", "", f"    {command}", "",
           "One context of the workload after its initialisation (warm-up and timed steps,",
           "captured CG iterations replayed as HIP graphs, then the profiled windows, kernels",
           "launched directly); durations are rocprofv3's",
           f"dispatch timestamps ({len(kt)} dispatches, span {span:.2f} ms, kernel time "
           f"{total / 1e3:.2f} ms).", "",
           "| kernel | calls | total ms | mean us | % |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:30]:
        out.append(f"| {k} | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.1f} | "
                   f"{100 * sum(v) / total:.1f} |")
    if workload == "config5":
        # bench.py's profiled windows close the run: every kernel class, the
        # dominant class alone (its event-timed launches give the roofline's
        # mean_launch_us), the surrogate alone; 3 steps each, k_stats ending
        # every step
        ends = [i for i, r in enumerate(kt) if name(r).startswith("k_stats")]
        if len(ends) >= 7:
            win = kt[ends[-7] + 1:ends[-4] + 1]
            wd = collections.defaultdict(list)
            for r in win:
                wd[name(r)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            out += ["", "The dominant-class window (the 3 steps bench.py times the dominant kernel "
                        "in, with HIP events on its launches; other classes run untimed).  Launches "
                        "that found every system finished (a few us: the replayed iteration pairs' "
                        "no-ops) are left out, as the library's timing leaves them out:", "",
                    "| kernel | launches | mean us |", "|---|---:|---:|"]
            for k, v in sorted(wd.items(), key=lambda kv: -sum(kv[1]))[:6]:
                real = [x for x in v if x >= 0.02 * max(v)]
                out.append(f"| {k} | {len(real)} | {sum(real) / len(real):.1f} |")
    open(os.path.join(ROOT, "profiles", f"{tag}_kernel_stats.md"), "w").write("\n".join(out) + "\n")

    def counters(folder):
        allr, ctx = stepped_context(one_csv(folder, "counter_collection.csv"), "Dispatch_Id")
        first = min(i for i, r in enumerate(allr) if "k_init_cells" in r["Kernel_Name"])
        copies = [float(r["Counter_Value"]) for r in allr[:first]
                  if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) > 100000]
        return ctx, copies
    F, cf = counters(f_dir)
    W, cw = counters(w_dir)
    ffac, wfac = COPY_KIB / (sum(cf) / len(cf)), COPY_KIB / (sum(cw) / len(cw))
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    table = ["| kernel | dispatches (all systems iterating) | FETCH B/voxel | WRITE B/voxel | "
             "measured B/voxel | algorithmic B/voxel | ratio |", "|---|---:|---:|---:|---:|---:|---:|"]
    ktimes = {}
    for full, (short, bpv) in ks.items():
        fd = [(int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in F if name(r) == full]
        wd = {int(r["Dispatch_Id"]): float(r["Counter_Value"]) for r in W if name(r) == full}
        if not fd:
            continue
        top = max(v for _, v in fd)
        full_disp = [(d, v) for d, v in fd if v >= 0.9 * top]   # every system still iterating
        # the all-systems dispatches of the FETCH pass; WRITE of the same dispatch order
        fetch = sum(v for _, v in full_disp) / len(full_disp) * 1024 * ffac
        wvals = sorted(wd.values(), reverse=True)[:len(full_disp)]
        write = sum(wvals) / len(wvals) * 1024 * wfac
        vox = 3 * nvox * nrep
        mb = (fetch + write) / vox
        durs = [x for x in dur.get(full, [])]
        ktimes[short] = durs
        rec = {"kernel": short, "workload": workload, "precision": int(precision), "sources": SOURCES,
               "sources_sha256": h.hexdigest(), "fetch_factor": ffac, "write_factor": wfac,
               "voxels_all_systems": vox, "dispatches_all_systems": len(full_disp),
               "fetch_bytes_per_voxel": fetch / vox, "write_bytes_per_voxel": write / vox,
               "traffic_bytes_per_voxel": mb, "algorithmic_bytes_per_voxel": bpv,
               "commands": [pmc_command(command, "FETCH_SIZE"), pmc_command(command, "WRITE_SIZE")]}
        json.dump(rec, open(os.path.join(ROOT, "profiles", f"{short}_{tag}_traffic.json"), "w"), indent=1)
        table.append(f"| {full} | {len(full_disp)} | {fetch / vox:.2f} | {write / vox:.2f} | {mb:.2f} | "
                     f"{bpv:.1f} | {mb / bpv:.3f} |")
    small = ["| kernel | dispatches | mean us | FETCH KiB/dispatch | WRITE KiB/dispatch | GB/s |",
             "|---|---:|---:|---:|---:|---:|"]
    for full in PER_LAUNCH:
        fd = [float(r["Counter_Value"]) for r in F if name(r) == full]
        wd = [float(r["Counter_Value"]) for r in W if name(r) == full]
        du = dur.get(full, [])
        if not fd or not wd or not du:
            continue
        fk, wk, us = sum(fd) / len(fd) * ffac, sum(wd) / len(wd) * wfac, sum(du) / len(du)
        small.append(f"| {full} | {len(fd)} | {us:.1f} | {fk:.0f} | {wk:.0f} | "
                     f"{(fk + wk) * 1024 / (us * 1e-6) / 1e9:.0f} |")
    md = [f"# HBM traffic of the solver's streaming kernels: {tag}", "",
          "Commands (repository root, one MI355X), one counter per run:", "",
          "    " + pmc_command(command, "FETCH_SIZE"),
          "    " + pmc_command(command, "WRITE_SIZE"), "",
          "Calibration: `--copy-calibration 256` first copies 256 MiB device to device (the",
          f"runtime's blit kernel); per copy FETCH_SIZE reads {sum(cf) / len(cf):.0f} KiB and WRITE_SIZE",
          f"{sum(cw) / len(cw):.0f} KiB for {COPY_KIB} KiB moved each way: scale factors",
          f"{ffac:.3f} (fetch) and {wfac:.3f} (write).", "",
          f"Per voxel of all {3 * nrep} systems ({3 * nvox * nrep} voxels), on the dispatches where every",
          "system still iterates (counter within 10 % of the kernel's largest; later",
          "dispatches skip finished systems):", ""] + table + [
          "", "Kernels below level 0 (latency-bound: bytes per dispatch over all systems, mean",
          "duration from the kernel trace, effective rate):", ""] + small + [
          "", "`profiles/<kernel>_" + tag + "_traffic.json` hold these numbers with the SHA-256 of the",
          "solver's sources; `bench.py` reports them as `roofline.traffic` only while those",
          "sources are unchanged."]
    open(os.path.join(ROOT, "profiles", f"solver_{tag}_traffic.md"), "w").write("\n".join(md) + "\n")
    print(f"wrote profiles/{tag}_kernel_stats.md, profiles/solver_{tag}_traffic.md and the json records")


if __name__ == "__main__":
    if len(sys.argv) != 7:
        raise SystemExit(__doc__)
    main(*sys.argv[1:])
