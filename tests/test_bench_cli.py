"""The benchmark's command-line contract on the CPU: more than one GPU is refused with a
message (the multi-GPU decomposition is a design only), before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")      # no result line


def test_roofline_entry_fractions():
    """The roofline object of a temporally blocked launch: the scope's convention (K steps of
    single-step bytes per launch) beside the launch's own one-pass position under the roof;
    counter traffic only for a kernel whose record matches the current source."""
    sys.path.insert(0, ROOT)
    import bench
    cells, K, t = 4096 * 4096, 7, 180e-6
    r = bench.roofline_entry("no_such_kernel<float, 7>", t, 28 * cells * K, 28 * cells, 44)
    assert r["traffic"] is None and "frac_measured" not in r
    assert abs(r["achieved"] - 28 * cells * K / t / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-3
    assert abs(r["frac_one_pass"] - 28 * cells / t / 8e12) < 1e-3
    assert abs(r["one_pass_time_us"] - 28 * cells / 8e12 * 1e6) < 0.01
    assert r["frac_one_pass"] < 1.0 < r["frac"]


def test_measured_traffic_needs_every_named_source_unchanged(tmp_path, monkeypatch):
    """Counter traffic is used only while each source the record names hashes as it did when
    the counters were taken."""
    import hashlib
    import json
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_1903_12522_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "a.hip").write_text("kernel a")
    (csrc / "b.h").write_text("header b")
    sha = {n: hashlib.sha256((csrc / n).read_bytes()).hexdigest() for n in ("a.hip", "b.h")}
    rec = {"sources": sha, "kernels": {
        "k1": {"source": ["a.hip", "b.h"], "fetch_bytes_per_launch": 300,
               "write_bytes_per_launch": 100},
        "k2": {"source": "a.hip", "fetch_bytes_per_launch": 10, "write_bytes_per_launch": 5},
        "k3": {"fetch_bytes_per_launch": 1, "write_bytes_per_launch": 1},
        "k5 @ w1": {"source": "a.hip", "fetch_bytes_per_launch": 7, "write_bytes_per_launch": 1},
        "k5 @ w2": {"source": "a.hip", "fetch_bytes_per_launch": 9, "write_bytes_per_launch": 1}}}
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k1") == 400
    assert bench.measured_traffic("k2") == 15
    assert bench.measured_traffic("k3") is None       # no source recorded
    assert bench.measured_traffic("k4") is None       # no record
    assert bench.measured_traffic("k5", "w1") == 8    # one instance, two workloads
    assert bench.measured_traffic("k5", "w2") == 10
    assert bench.measured_traffic("k5", "w3") is None
    (csrc / "b.h").write_text("header b, edited")
    assert bench.measured_traffic("k1") is None       # one of its sources changed
    assert bench.measured_traffic("k2") == 15
