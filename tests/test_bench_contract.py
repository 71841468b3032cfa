"""bench.py's command-line contract on the CPU: it refuses more than one GPU
(or a multi-rank launch) with a message and exit status 2, before touching a
GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    r = _bench(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_multi_rank_launch_is_refused():
    r = _bench([], env=dict(os.environ, WORLD_SIZE="8"))
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
