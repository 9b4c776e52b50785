"""bench.py command line (no GPU needed): more than one GPU is refused with a
message, and the workload list is the documented one."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workloads_listed_in_help():
    r = run("--help")
    assert r.returncode == 0
    for c in ("batch", "pair", "allpairs", "ragged", "ragged_any", "bf16", "srv", "copy"):
        assert c in r.stdout


def test_per_workload_defaults_and_explicit_flags(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    for cfg, (steps, warmup) in bench.DEFAULT_STEPS.items():
        monkeypatch.setattr(sys, "argv", ["bench.py", "--config", cfg])
        a = bench.parse()
        assert (a.steps, a.warmup) == (steps, warmup)
        assert warmup >= 10 and steps >= 40
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "7", "--warmup", "2"])
    a = bench.parse()
    assert (a.steps, a.warmup, a.config) == (7, 2, "batch")
