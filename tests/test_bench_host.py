"""Host logic of bench.py (no GPU): the one-GPU rule, the HBM byte arithmetic
of the traffic record from rocprofv3 counter CSVs, and the rule that a record
taken from other kernel sources is not reported."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fp:
        w = csv.DictWriter(fp, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for row in rows:
            name, value = row[:2]
            grid = row[2] if len(row) > 2 else 64
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_bytes_from_counters(tmp_path):
    fp64 = bench.TRAFFIC_KERNELS["gain_binned_fp64_3d_n32"][0] + "(pgc::GainParams<double>, pgc::BinItems)"
    other = "void pgc::(anonymous namespace)::sep_apply<double>(...)"
    copy = "__amd_rocclr_copyBuffer"
    d = str(tmp_path)
    # two dispatches of the gain (the mean is used) and an unrelated kernel
    _counter_csv(os.path.join(d, "f.csv"), "FETCH_SIZE", [(fp64, 1000.0), (fp64, 3000.0), (other, 5.0)])
    _counter_csv(os.path.join(d, "w.csv"), "WRITE_SIZE", [(fp64, 100.0), (fp64, 100.0), (other, 1.0)])
    # a 1 GiB copy reads FETCH_SIZE = 2^19 KiB and writes WRITE_SIZE = 2^20 KiB
    _counter_csv(os.path.join(d, "cf.csv"), "FETCH_SIZE", [(copy, float(1 << 19)), (copy, float(1 << 19))])
    _counter_csv(os.path.join(d, "cw.csv"), "WRITE_SIZE", [(copy, float(1 << 20))])
    out = os.path.join(d, "traffic.json")
    rec = bench.write_traffic(*(os.path.join(d, n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")), path=out)
    e = rec["gain_binned_fp64_3d_n32"]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    # (2000 KiB x 2 + 100 KiB x 1) x 1024 bytes
    assert e["bytes_per_launch"] == 1024.0 * (2000.0 * 2.0 + 100.0)
    assert set(rec) == {"gain_binned_fp64_3d_n32"}
    assert json.load(open(out)) == rec
    assert bench.traffic_for("gain_binned_fp64_3d_n32", path=out) == e["bytes_per_launch"]
    assert bench.traffic_for("gain_batched_lanes_2d_4096", path=out) is None


def test_traffic_counts_the_largest_grid_of_a_kernel(tmp_path):
    """The profile run also launches the gain per chunk of a streamed index,
    on smaller grids: only the dispatches of the largest grid are averaged."""
    fp64 = bench.TRAFFIC_KERNELS["gain_binned_fp64_3d_n32"][0] + "(pgc::GainParams<double>, pgc::BinItems)"
    path = os.path.join(str(tmp_path), "f.csv")
    _counter_csv(path, "FETCH_SIZE", [(fp64, 1000.0, 9000), (fp64, 3000.0, 9000), (fp64, 10.0, 5000),
                                      (fp64, 12.0, 4000)])
    assert bench.counter_per_dispatch(path, "FETCH_SIZE") == {fp64: 2000.0}


def test_traffic_of_other_sources_is_not_reported(tmp_path):
    out = os.path.join(str(tmp_path), "traffic.json")
    rec = {"gain_binned_fp64_3d_n32": {"kernel_source_sha256": "0" * 64, "bytes_per_launch": 1.0}}
    json.dump(rec, open(out, "w"))
    assert bench.traffic_for("gain_binned_fp64_3d_n32", path=out) is None
    rec["gain_binned_fp64_3d_n32"]["kernel_source_sha256"] = bench.sources_sha("gain_binned")
    json.dump(rec, open(out, "w"))
    assert bench.traffic_for("gain_binned_fp64_3d_n32", path=out) == 1.0
    assert bench.traffic_for("no_such_kernel", path=out) is None
    assert bench.traffic_for("gain_binned_fp64_3d_n32", path=os.path.join(str(tmp_path), "missing.json")) is None


def test_committed_traffic_record():
    """The committed record covers every profiled kernel with positive byte
    counts; a record taken from other kernel sources is reported as a skip
    (bench.py then prints traffic as null until the counters are taken again)."""
    rec = json.load(open(bench.TRAFFIC_PATH))
    stale = []
    for tag, (prefix, kind) in bench.TRAFFIC_KERNELS.items():
        assert tag in rec
        assert rec[tag]["kernel"] == prefix
        assert rec[tag]["bytes_per_launch"] > 0
        if rec[tag]["kernel_source_sha256"] != bench.sources_sha(kind):
            stale.append(tag)
    if stale:
        pytest.skip("traffic record predates the current sources of: " + ", ".join(stale))


def _golden(name):
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", name))
            if l.strip() and not l.startswith("#")]
    return rows


def test_accuracy_tables_match_the_golden_files():
    """The accuracy study's copies of Tables 2 and 3 are the cited golden values."""
    for map_ in (0, 1):
        rows = _golden("table2_bkw2d_cheb%d.txt" % map_)
        assert [int(r[0]) for r in rows] == list(bench.TABLE2_DEGREES)
        assert [float(r[2]) for r in rows] == bench.TABLE2_BEST_L2[map_]
    rows = _golden("table3_bkw3d_cheb0.txt")
    assert {int(r[0]): (int(r[2]), float(r[3])) for r in rows} == bench.TABLE3_LINF
