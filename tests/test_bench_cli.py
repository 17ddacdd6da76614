"""bench.py's command-line contract on the host (no GPU needed): it runs on
one GPU only and says so for any other count, and it documents its modes."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_measurement_modes():
    r = run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--c2-to-tol", "--poisson-only",
                 "--batch-cap", "--copy-calibration", "--qr-micro-only"):
        assert flag in r.stdout, flag


def test_cpu_baseline_leg_runs_on_a_small_sample():
    """The CPU-baseline leg (the oracle timed on the host) on a small basis:
    every add of its timing loop must be accepted (each cycle adds a fresh
    column, since the delete drops the oldest one)."""
    sys.path.insert(0, ROOT)
    import bench
    out = bench.cpu_baseline(n=1 << 12, k=5, reps=3, c2_s=12, c2_m=4, c2_iters=2)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["one_core_value"] > 0
    assert out["cores"] >= 1
    c2 = out["c2_iteration_all_cores"]
    assert c2["ms_per_iteration"] > 0 and c2["threads"] >= 1 and c2["timed_iterations"] == 2
