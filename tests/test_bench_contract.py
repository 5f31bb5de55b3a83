"""bench.py's traffic figure: taken from the committed rocprofv3 counter
passes only while the step kernel's sources are the ones that were profiled."""
import hashlib
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_profile(path, sources, kernel="k_fused<1, 2, double>"):
    rec = {"kernel": kernel, "sources": sources, "dispatches": 2,
           "fetch_kib_per_dispatch": 1000.0, "write_kib_per_dispatch": 10.0,
           "copy_bytes": 1 << 20, "copy_fetch_kib": 512.0, "copy_write_kib": 1024.0}
    with open(path, "w") as f:
        f.write("# summary\n\n```json kpp-traffic\n" + json.dumps(rec) + "\n```\n")


def test_traffic_scaled_by_copy_calibration(tmp_path):
    bench = load_bench()
    rel = "paper_2501_11673_amd/csrc/fused.hip"
    digest = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()
    prof = tmp_path / "p.md"
    write_profile(prof, {rel: digest})
    # FETCH read 512 KiB for a 1 MiB copy (x2), WRITE read 1024 KiB (x1)
    assert bench.measured_traffic(str(prof), "k_fused<1, 2, double>") == 1000.0 * 2048 + 10.0 * 1024
    assert bench.measured_traffic(str(prof), "k_fused<1, 1, double>") is None


def test_traffic_dropped_when_kernel_changed(tmp_path):
    bench = load_bench()
    prof = tmp_path / "p.md"
    write_profile(prof, {"paper_2501_11673_amd/csrc/fused.hip": "0" * 64})
    assert bench.measured_traffic(str(prof), "k_fused<1, 2, double>") is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), "k_fused<1, 2, double>") is None
    assert bench.measured_traffic(None, "k_fused<1, 2, double>") is None
