"""Summaries of rocprofv3 runs of the plain 128^3 bench workload.

Reads three rocprofv3 output folders of the same command (a kernel trace,
a FETCH_SIZE pass and a WRITE_SIZE pass, each started with
`--copy-calibration 256` so that the runtime's copy of 256 MiB calibrates the
counters) and writes, under profiles/:

  plain128_kernel_stats.md                per-kernel durations of the timed context
  <kernel>_plain128_traffic.{json,md}     HBM bytes per launch of the CG kernels

Usage: python -m paper_2105_00448_amd.profile_summary KT_DIR FETCH_DIR WRITE_DIR BENCH_JSON COMMAND
"""
import collections
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["paper_2105_00448_amd/csrc/k_solver.hip", "paper_2105_00448_amd/csrc/dev_util.h",
           "paper_2105_00448_amd/csrc/hca_internal.h"]
KERNELS = {"k_cg_apply": "k_cg_apply<false>", "k_cg_update": "k_cg_update<false>"}
COPY_KIB = 256 * 1024


def name(r):
    return r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hca::", "")


def one_csv(folder, suffix):
    hits = glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)
    if len(hits) != 1:
        raise SystemExit(f"expected one *{suffix} under {folder}, found {hits}")
    return list(csv.DictReader(open(hits[0])))


def timed_context(rows, key):
    """Dispatches after the last context initialisation (k_init_cells)."""
    rows = sorted(rows, key=lambda r: int(r[key]))
    last = max(i for i, r in enumerate(rows) if "k_init_cells" in r["Kernel_Name"])
    return rows, rows[last + 1:]


def main(kt_dir, f_dir, w_dir, bench_json, command):
    bench = json.load(open(bench_json))
    _, kt = timed_context(one_csv(kt_dir, "kernel_trace.csv"), "Start_Timestamp")
    dur = collections.defaultdict(list)
    for r in kt:
        dur[name(r)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in dur.values())
    span = (int(kt[-1]["End_Timestamp"]) - int(kt[0]["Start_Timestamp"])) / 1e6
    out = [f"# Kernel statistics: plain 128^3 workload (multigrid-preconditioned CG)", "",
           "Command (repository root, one MI355X):", "", f"    {command}", "",
           "The bench's plain leg: one timed repeat (100 coupled steps, captured CG",
           "iterations replayed as HIP graphs), then one more repeat in a fresh context",
           "with start/stop events carried by the launches of the dominant kernel (every",
           "kernel launched directly there).  Durations are rocprofv3's dispatch",
           "timestamps over that last context, after its initialisation",
           f"({len(kt)} dispatches, span {span:.2f} ms, kernel time {total / 1e3:.2f} ms).", "",
           "| kernel | calls | total ms | mean us | % |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:26]:
        out.append(f"| {k} | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.1f} | {100 * sum(v) / total:.1f} |")
    rl = bench.get("roofline", {})
    out += ["", f"Bench line of this traced run: {bench['ms_per_step']:.3f} ms per step; roofline kernel "
            f"`{rl.get('kernel')}`, {rl.get('mean_launch_us', 0):.1f} us per launch from HIP events "
            f"({rl.get('launches')} launches, {rl.get('bytes_per_launch', 0) / 1e6:.1f} MB algorithmic each)."]
    for short, full in KERNELS.items():
        v = [x for x in dur.get(full, []) if x > 10.0]
        if v:
            out.append(f"rocprofv3 `{full}`: {len(v)} working dispatches (> 10 us; the others found every "
                       f"system finished), mean {sum(v) / len(v):.1f} us.")
    out += ["", "Under the tracer the HIP events read a few microseconds above the dispatch",
            "timestamps of the same launches; the untraced bench's events for the roofline",
            "kernel are the figure to compare with the working-dispatch mean above."]
    open(os.path.join(ROOT, "profiles", "plain128_kernel_stats.md"), "w").write("\n".join(out) + "\n")

    def counters(folder):
        allr, ctx = timed_context(one_csv(folder, "counter_collection.csv"), "Dispatch_Id")
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
    bpv = {"k_cg_apply": 36.0, "k_cg_update": 56.0}
    nvox = 3 * 128 ** 3
    for short, full in KERNELS.items():
        fa = [float(r["Counter_Value"]) for r in F if name(r) == full]
        wa = [float(r["Counter_Value"]) for r in W if name(r) == full]
        act = [x for x in fa if x > 1024.0]   # all-finished dispatches read almost nothing
        n = len(act)
        fetch = sum(fa) * 1024 * ffac / n
        write = sum(wa) * 1024 * wfac / n
        rec = {"kernel": short, "workload": "plain128", "sources": SOURCES, "sources_sha256": h.hexdigest(),
               "fetch_factor": ffac, "write_factor": wfac, "fetch_bytes_per_launch": fetch,
               "write_bytes_per_launch": write, "traffic_bytes_per_launch": fetch + write, "launches": n,
               "command": command.replace("--kernel-trace --stats", "--pmc FETCH_SIZE|WRITE_SIZE")}
        json.dump(rec, open(os.path.join(ROOT, "profiles", f"{short}_plain128_traffic.json"), "w"), indent=1)
        md = [f"# HBM traffic of {short} on the plain 128^3 workload", "",
              "Commands (repository root, one MI355X), one counter per run:", "",
              "    " + command.replace("--kernel-trace --stats", "--pmc FETCH_SIZE").replace("P_kt", "P_f"),
              "    " + command.replace("--kernel-trace --stats", "--pmc WRITE_SIZE").replace("P_kt", "P_w"), "",
              f"Calibration: `--copy-calibration 256` first copies 256 MiB device to device (runtime",
              f"blit kernel); per copy FETCH_SIZE reads {sum(cf) / len(cf):.0f} KiB and WRITE_SIZE",
              f"{sum(cw) / len(cw):.0f} KiB for {COPY_KIB} KiB moved each way: scale factors",
              f"{ffac:.3f} (fetch) and {wfac:.3f} (write).", "",
              f"{full}, dispatches of the timed context, averaged over the {n} dispatches",
              "with at least one system iterating (all-finished dispatches read almost nothing",
              "and are summed in, not counted):", "",
              "| quantity | per launch |", "|---|---:|",
              f"| FETCH_SIZE x {ffac:.3f} | {fetch / 1e6:.1f} MB |",
              f"| WRITE_SIZE x {wfac:.3f} | {write / 1e6:.1f} MB |",
              f"| traffic | {(fetch + write) / 1e6:.1f} MB |",
              f"| algorithmic, all three systems iterating ({bpv[short]:.0f} B x {nvox} voxels) | "
              f"{bpv[short] * nvox / 1e6:.1f} MB |", "",
              f"`profiles/{short}_plain128_traffic.json` holds these numbers with the SHA-256 of the",
              "kernel's source files; `bench.py` reports them as `roofline.traffic` only while",
              "those sources are unchanged."]
        open(os.path.join(ROOT, "profiles", f"{short}_plain128_traffic.md"), "w").write("\n".join(md) + "\n")
    print("wrote profiles/plain128_kernel_stats.md and the traffic summaries")


if __name__ == "__main__":
    if len(sys.argv) != 6:
        raise SystemExit(__doc__)
    main(*sys.argv[1:])
