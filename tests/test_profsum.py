"""Host logic of the profile summaries (CPU): copy-calibrated HBM bytes,
per-schedule counter records, the comment-insensitive scan source hash, the
unit-activity figures, and that the committed counter record was taken on
the scan sources as they stand."""
import csv
import importlib.util
import json
import os

import pytest

from paper_1306_1467_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, (kernel, counter, value, t0, t1) in enumerate(rows):
            r = {f: 0 for f in FIELDS}
            r.update({"Dispatch_Id": k + 1, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value,
                      "Start_Timestamp": t0, "End_Timestamp": t1})
            w.writerow(r)
    return str(path)


COPY = "__amd_rocclr_copyBuffer"
SCAN = "void vjb::k_scan<3, true, 512, 4, 16, true>(vjb::JobDev, HIP_vector_type<double, 2u>*)"


def test_counters_are_scaled_by_the_copy(tmp_path):
    gib = 4
    # the copy reads 4 GiB: FETCH_SIZE counts half of it, WRITE_SIZE all of it (KiB)
    fetch = _csv(tmp_path / "f.csv", [(COPY, "FETCH_SIZE", 2 * 2 ** 20, 0, 1), (SCAN, "FETCH_SIZE", 1000.0, 0, 1),
                                      (SCAN, "FETCH_SIZE", 3000.0, 0, 1)])
    write = _csv(tmp_path / "w.csv", [(COPY, "WRITE_SIZE", 4 * 2 ** 20, 0, 1), (SCAN, "WRITE_SIZE", 10.0, 0, 1)])
    out = tmp_path / "rec.json"
    text = profsum.counters(fetch, write, gib, r"k_scan<3, true, 512, 4, 16, true>", "fp32_wide", 9, "cf", "cw",
                            str(out), 4096000)
    doc = json.load(open(out))
    assert len(doc["records"]) == 1
    rec = doc["records"][0]
    r9 = rec["schedules"]["9"]
    # mean fetch 2000 KiB at 0.5 counter bytes per byte -> 4,096,000 bytes; write 10 KiB at 1.0
    assert r9["fetch_bytes_per_launch"] == 4096000
    assert r9["write_bytes_per_launch"] == 10240
    assert r9["bytes_per_launch"] == 4106240
    assert r9["launches"] == [2, 1]
    assert rec["scan_source_hash"] == profsum.scan_source_hash() and rec["precision"] == "fp32_wide"
    assert "measured / algorithmic = 1.0025" in text
    # a second schedule is added beside the first; another precision gets a record of its own
    profsum.counters(fetch, write, gib, r"k_scan<3, true, 512, 4, 16, true>", "fp32_wide", 3, "cf", "cw", str(out),
                     None)
    assert sorted(json.load(open(out))["records"][0]["schedules"]) == ["3", "9"]
    profsum.counters(fetch, write, gib, r"k_scan<3, true, 512, 4, 16, true>", "fp64", 3, "cf", "cw", str(out), None)
    recs = {r["precision"]: r for r in json.load(open(out))["records"]}
    assert sorted(recs) == ["fp32_wide", "fp64"] and sorted(recs["fp64"]["schedules"]) == ["3"]
    # a record of other scan sources is dropped
    doc = json.load(open(out))
    doc["records"][0]["scan_source_hash"] = "stale"
    json.dump(doc, open(out, "w"))
    profsum.counters(fetch, write, gib, r"k_scan<3, true, 512, 4, 16, true>", "fp64", 9, "cf", "cw", str(out), None)
    recs = {r["precision"]: r for r in json.load(open(out))["records"]}
    assert sorted(recs) == ["fp64"] and sorted(recs["fp64"]["schedules"]) == ["3", "9"]


def test_counters_need_the_copy_and_the_kernel(tmp_path):
    no_copy = _csv(tmp_path / "a.csv", [(SCAN, "FETCH_SIZE", 1.0, 0, 1)])
    with pytest.raises(SystemExit):
        profsum.counters(no_copy, no_copy, 4, "k_scan", "fp32_wide", 0, "", "", None, None)
    no_scan = _csv(tmp_path / "b.csv", [(COPY, "FETCH_SIZE", 1.0, 0, 1)])
    with pytest.raises(SystemExit):
        profsum.counters(no_scan, no_scan, 4, "k_scan", "fp32_wide", 0, "", "", None, None)


def test_source_hash_ignores_comments_only():
    code = "int f(int a) {\n    return a + 1;   // one more\n}\n/* block\n comment */\n"
    assert profsum._code_only(code) == profsum._code_only("int f(int a) { return a + 1; }")
    assert profsum._code_only(code) != profsum._code_only("int f(int a) { return a + 2; }")


def test_activity_figures(tmp_path):
    # 2 dispatches of 1 ms; GRBM_GUI_ACTIVE summed over 8 XCDs = 8 * 2.4e6 cycles -> 2.4 GHz
    keys = 64 * 1000
    rows = []
    for d in range(2):
        rows += [(SCAN, "GRBM_GUI_ACTIVE", 8 * 2.4e6, 0, 1_000_000), (SCAN, "SQ_INSTS_VALU", 7000.0, 0, 1_000_000),
                 (SCAN, "SQ_INSTS_LDS", 1000.0, 0, 1_000_000),
                 (SCAN, "SQ_LDS_BANK_CONFLICT", 256 * 1.2e6, 0, 1_000_000)]
    text = profsum.activity([_csv(tmp_path / "s.csv", rows)], r"k_scan<", keys, ["cmd"])
    assert "Clock (busy cycles per XCD / dispatch duration, median over dispatches): 2.40 GHz" in text
    assert "VALU instructions per key (wave-wide): 7.00" in text
    assert "LDS instructions per key (wave-wide): 1.00" in text
    assert "LDS bank-conflict cycles per CU / busy cycles: 0.50" in text


def test_committed_counter_record_matches_the_scan_sources():
    """bench.py reports traffic only from a record taken on the current scan
    code: a record whose source hash matches is used as committed, a stale
    one never."""
    path = os.path.join(ROOT, "profiles", "stump_scan_faces15k_counters.json")
    doc = json.load(open(path))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    precisions = set()
    for rec in doc.get("records", [doc]):
        current = rec["scan_source_hash"] == profsum.scan_source_hash()
        precisions.add(rec["precision"])
        for s, r in rec["schedules"].items():
            got = bench.profiled_traffic("faces15k", rec["precision"], int(s))
            if current:
                assert got == r["bytes_per_launch"]
                assert 1.0 <= r["bytes_per_launch"] / 4870080000 < 1.01
            else:
                assert got is None
    other = next(p for p in ("fp64", "fp32", "fp32_wide", "fp32_kahan") if p not in precisions)
    assert bench.profiled_traffic("faces15k", other, 9) is None
