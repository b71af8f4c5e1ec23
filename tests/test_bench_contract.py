"""bench.py's command-line contract on the CPU: runs above one GPU are refused
before anything touches a device (the library has no multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, env=e, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 1" in r.stderr
    assert r.stdout == ""                     # no JSON line


def test_a_multi_rank_launch_is_refused():
    r = _bench("--steps", "1", env={"WORLD_SIZE": "4"})
    assert r.returncode == 2 and "one GPU only" in r.stderr
