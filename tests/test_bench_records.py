"""The profile records bench.py reads (HBM byte counters, VALU instruction counts): each
names the command that made it, applies only to its kernel, launch shape, stream structure,
workload and precision, and only while the kernel sources hash to the recorded value."""

import glob
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_counters_*.json")) +
                 glob.glob(os.path.join(ROOT, "profiles", "sq_counters_*.json")))


def test_records_exist():
    assert any("hbm_counters_stage_terms_shear8192" in r for r in RECORDS)
    assert any("sq_counters_stage_terms_shear8192" in r for r in RECORDS)


@pytest.mark.parametrize("path", RECORDS, ids=os.path.basename)
def test_record_fields_and_commands(path):
    rec = json.load(open(path))
    for k in ("kernel_class", "kernel", "tile_rows", "threads", "workload", "precision",
              "sources", "source_sha256", "commands"):
        assert k in rec, k
    for cmd in rec["commands"]:
        assert cmd.startswith("cd /tmp && export TMPDIR=/tmp") and "rocprofv3 --pmc" in cmd
        assert "bench.py" in cmd
    for src in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, src)), src


def test_current_records_apply_only_to_their_conditions():
    rec = json.load(open(os.path.join(ROOT, "profiles",
                                      "hbm_counters_stage_terms_shear8192_fp32split.json")))
    shape = (rec["tile_rows"], rec["threads"])
    st = rec.get("structure", 0)
    got = bench.recorded_traffic(rec["kernel_class"], rec["workload"], rec["precision"], shape, st)
    assert got == rec["traffic_bytes_per_launch"]
    other = 0 if st == 2 else 2
    assert bench.recorded_traffic(rec["kernel_class"], rec["workload"], rec["precision"], shape,
                                  other) is None
    assert bench.recorded_traffic(rec["kernel_class"], rec["workload"], "fp64", shape, st) is None
    assert bench.recorded_traffic(rec["kernel_class"], rec["workload"], rec["precision"],
                                  (shape[0], 256 if shape[1] == 512 else 512), st) is None
    srec = json.load(open(os.path.join(ROOT, "profiles",
                                       "sq_counters_stage_terms_shear8192_fp32split.json")))
    v = bench.recorded_valu_issue_us(srec["kernel_class"], srec["workload"], srec["precision"],
                                     (srec["tile_rows"], srec["threads"]), srec["structure"])
    assert v == srec["valu_issue_us_per_launch"] and v > 0
