"""bench.py's command line on the host (no GPU): it measures one GPU only and
says so when asked for more, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300, env=env)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_a_multi_rank_launch_is_refused_too():
    env = dict(os.environ, WORLD_SIZE="4")
    r = _bench(env=env)
    assert r.returncode == 2 and "WORLD_SIZE 4" in r.stderr


def test_help_lists_the_workloads():
    r = _bench("--help")
    assert r.returncode == 0
    for w in ("--workload", "--steps", "--warmup", "--gpus"):
        assert w in r.stdout
