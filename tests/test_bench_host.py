"""Host-side logic of bench.py: the rocprofv3 counter summary behind
roofline.traffic and its staleness check (no GPU use)."""
import csv
import importlib.util
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_summary_calibrates_and_detects_stale_sources(tmp_path, monkeypatch):
    bench = load_bench()
    src = tmp_path / "ctr"
    # the 1 GiB copy reads half its bytes in FETCH_SIZE KiB (factor 2) and writes all of them
    write_counters(str(src / "fetch"), "FETCH_SIZE",
                   [("__amd_rocclr_copyBuffer", 524288), ("__amd_rocclr_copyBuffer", 4),
                    ("void ccm::mv::k_matvec_al<3, false>(x)", 1000),
                    ("void ccm::mv::k_matvec_w<17, true>(x)", 3000)])
    write_counters(str(src / "write"), "WRITE_SIZE",
                   [("__amd_rocclr_copyBuffer", 1048576),
                    ("void ccm::mv::k_matvec_al<3, false>(x)", 128),
                    ("void ccm::mv::k_matvec_w<17, true>(x)", 128)])
    out = tmp_path / "summary.md"
    bench.summarize_counters(str(src), str(out))
    text = out.read_text()
    # bytes = KiB * 1024 * factor: (1000*2 + 128) KiB and (3000*2 + 128) KiB
    assert "| 2179072 |" in text and "| 6275072 |" in text
    assert "HBM bytes per launch (mean over the sweep): 4227072" in text
    monkeypatch.setattr(bench, "COUNTERS_MD", str(out))
    assert bench.recorded_traffic() == 4227072.0
    # a change of the matvec sources makes the recorded counters stale
    monkeypatch.setattr(bench, "matvec_source_hash", lambda: "0" * 16)
    assert bench.recorded_traffic() is None


def test_gpus_other_than_one_exit_with_message():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stdout
