"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the
comment-insensitive source hash that ties stored counters to the code, and
the fused Taylor update's profile summarizer on synthetic rocprofv3 files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_code_only_drops_comments_and_keeps_strings():
    src = ('int a = 1;  // trailing\n/* block\n   comment */ const char *s = "x // y /* z */";\n'
           "char q = '\"'; int b = 2; /* last */\n")
    assert bench._code_only(src) == 'int a = 1; const char *s = "x // y /* z */"; char q = \'"\'; int b = 2;'
    # a comment-only edit and re-indentation leave the code text unchanged
    assert bench._code_only(src.replace("trailing", "other words").replace("int b", "   int b")) == \
        bench._code_only(src)
    # a code edit does not
    assert bench._code_only(src.replace("int b = 2", "int b = 3")) != bench._code_only(src)


def test_kernel_template_arguments():
    name = "void hs::dia_tile_kernel<float, 1, 8, false, true, 1024, false, true>(hs::TileArgs)"
    assert bench._template_args(name) == ["float", "1", "8", "false", "true", "1024", "false", "true"]


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_taylor_summary_from_synthetic_profiles(tmp_path, monkeypatch):
    horner = "void hs::dia_tile_kernel<float, 1, 8, false, true, 1024, false, true>(hs::TileArgs)"
    other = "void hs::dia_tile_kernel<float, 1, 8, false, false, 1024, false, true>(hs::TileArgs)"
    rows = [{"workload": "small", "taylor_terms": 2, "h_diagonals": 3, "gb_per_stage": 1.0, "dispatches": 2},
            {"workload": "large", "taylor_terms": 1, "h_diagonals": 5, "gb_per_stage": 4.0, "dispatches": 2}]
    log = tmp_path / "leg.log"
    log.write_text("profiler chatter\n" + json.dumps({"leg": "taylor", "result": rows}) + "\n")
    # dispatch ids out of order on purpose; a non-Horner launch in between
    disp = [(3, horner, 300.0, 30.0, 2000, 2400), (1, horner, 100.0, 10.0, 1000, 1100), (2, other, 9.0, 9.0, 0, 1),
            (4, horner, 500.0, 50.0, 3000, 3600), (5, horner, 700.0, 70.0, 4000, 4800)]
    for d, cname, col in (("fetch", "FETCH_SIZE", 2), ("write", "WRITE_SIZE", 3)):
        os.makedirs(tmp_path / d)
        _write_csv(tmp_path / d / "run_counter_collection.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                                                "Counter_Value"],
                   [(i, k, cname, r[col]) for r in disp for i, k in [(r[0], r[1])]])
    os.makedirs(tmp_path / "trace")
    _write_csv(tmp_path / "trace" / "run_kernel_trace.csv", ["Dispatch_Id", "Kernel_Name", "Start_Timestamp",
                                                             "End_Timestamp"],
               [(r[0], r[1], r[4] * 1000, r[5] * 1000) for r in disp])
    _write_csv(tmp_path / "trace" / "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "MinNs", "MaxNs",
                                                             "Percentage"],
               [(horner, 4, 400000, 100000, 800000, 99.0)])
    cal = tmp_path / "traffic.json"
    cal.write_text(json.dumps({"fetch_scale": 2.0, "write_scale": 1.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(cal))
    monkeypatch.setattr(bench, "OUT_DIR", str(tmp_path))
    bench.summarize_taylor_profiles(str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"),
                                    str(log))
    md = (tmp_path / "dia_tile_horner_tfim_n24_n26.md").read_text()
    table = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:-1]]
             for l in md.splitlines() if l.startswith("| small") or l.startswith("| large")}
    # dispatches 1, 3 -> "small"; 4, 5 -> "large" (sorted by id, the other kernel skipped)
    # small: ms (0.1, 0.4) -> 0.25; fetch (100, 300) -> 200 KiB; write (10, 30) -> 20 KiB
    assert table["small"][:3] == ["0.250", "200", "20"]
    assert float(table["small"][3]) == pytest.approx((200 * 2.0 + 20 * 1.0) * 1024 / 1e9, abs=5e-4)
    assert table["small"][4] == "1.000"
    # large: ms (0.6, 0.8) -> 0.7; algorithmic 4 GB / 0.7 ms = 5714 GB/s
    assert table["large"][0] == "0.700" and table["large"][5] == "5714"
    assert "--summarize-taylor-profiles" in md


def test_taylor_summary_rejects_mismatched_dispatch_counts(tmp_path, monkeypatch):
    horner = "void hs::dia_tile_kernel<float, 1, 8, false, true, 1024, false, false>(hs::TileArgs)"
    log = tmp_path / "leg.log"
    log.write_text(json.dumps({"leg": "taylor", "result": [{"workload": "w", "taylor_terms": 1, "h_diagonals": 1,
                                                            "gb_per_stage": 1.0, "dispatches": 3}]}) + "\n")
    for d, cname in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        os.makedirs(tmp_path / d)
        _write_csv(tmp_path / d / "run_counter_collection.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                                                "Counter_Value"], [(1, horner, cname, 1.0)])
    os.makedirs(tmp_path / "trace")
    _write_csv(tmp_path / "trace" / "run_kernel_trace.csv", ["Dispatch_Id", "Kernel_Name", "Start_Timestamp",
                                                             "End_Timestamp"], [(1, horner, 0, 1000)])
    _write_csv(tmp_path / "trace" / "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "MinNs", "MaxNs",
                                                             "Percentage"], [])
    cal = tmp_path / "traffic.json"
    cal.write_text(json.dumps({"fetch_scale": 2.0, "write_scale": 1.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(cal))
    monkeypatch.setattr(bench, "OUT_DIR", str(tmp_path))
    with pytest.raises(SystemExit, match="dispatch counts differ"):
        bench.summarize_taylor_profiles(str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"),
                                        str(log))
