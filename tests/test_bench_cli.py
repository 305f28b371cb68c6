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
