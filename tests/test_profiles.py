"""The committed rocprofv3 summaries under profiles/ describe the current
solver: every HBM-traffic record names the sources it was measured with and
their SHA-256, which must match the files in the tree (the bench reports a
record's traffic only while they do), and the bench finds a record for the
kernels its headline and 128^3 lines report.  A failure here means the
solver changed after the counters were taken: rerun the rocprofv3 commands
written in the records and `python -m paper_2105_00448_amd.profile_summary`."""
import glob
import hashlib
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")))


def test_there_are_traffic_records():
    assert len(RECORDS) >= 8


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_traffic_record_matches_the_sources(path):
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    assert h.hexdigest() == rec["sources_sha256"], os.path.basename(path)
    assert rec["traffic_bytes_per_voxel"] > 0 and rec["algorithmic_bytes_per_voxel"] > 0
    for cmd in rec["commands"]:
        assert "bench.py" in cmd and "--pmc" in cmd


@pytest.mark.parametrize("kernel,workload", [("k_cg_apply", "config5"), ("k_mg_postfused_L0", "config5"),
                                             ("k_cg_apply", "config5_fp32"),
                                             ("k_mg_postfused_L0", "config5_fp32"),
                                             ("k_cg_apply", "plain128"),
                                             ("k_mg_postfused_L0", "plain128")])
def test_bench_reads_the_traffic(kernel, workload):
    assert bench.measured_traffic(kernel, workload, 1.0e9) is not None
