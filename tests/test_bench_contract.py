"""bench.py's output contract, checked on the host: the fields of the JSON
line and of its roofline object, the traffic figure taken only from a
counter summary of the same kernel source, and the refusal of more than
one GPU."""
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_line_and_roofline_fields():
    prof = {"onesweep": (4, 2.0), "hist": (1, 0.3)}
    roof = bench.hbm_roofline(prof, "onesweep", 2 * (1 << 28) * 4, traffic=123)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["avg_launch_ms"] - 0.5) < 1e-12
    assert abs(roof["achieved"] - 2 * (1 << 28) * 4 / 0.5e-3 / 1e9) < 1e-6
    assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-12 and roof["traffic"] == 123
    args = types.SimpleNamespace(steps=7, warmup=2)
    res = bench.line(args, 90.0, 3.0, "u32", "synthetic", {"workload": "w"}, roof, prof, {"x": 1})
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in res, k
    assert res["n_gpus"] == 1 and res["steps"] == 7 and res["warmup"] == 2 and res["x"] == 1
    assert res["higher_is_better"] is True and res["vs_baseline"] is None
    assert res["kernels"]["onesweep"] == {"launches": 4, "avg_ms": 0.5}
    # a kernel that never ran gives no rate rather than a made-up one
    empty = bench.hbm_roofline({}, "onesweep", 1)
    assert empty["achieved"] is None and empty["frac"] is None


def test_traffic_needs_the_same_kernel_source(tmp_path, monkeypatch):
    h = bench.source_hash(["rs_lsd.hip", "rs_dev.h"])
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    (prof_dir / "pmc_k_w.txt").write_text("source_sha256: %s\nhbm_bytes_per_launch: 4242\n" % h)
    (prof_dir / "pmc_k_old.txt").write_text("source_sha256: %s\nhbm_bytes_per_launch: 1\n" % ("0" * 64))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.pmc_traffic("k", "w", h) == 4242
    assert bench.pmc_traffic("k", "old", h) is None       # counters of another source
    assert bench.pmc_traffic("k", "missing", h) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
