"""bench.py's command line on the CPU: the multi-GPU request is refused with a
message (one GPU is measured), and the options parse."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--fmt", "--workload", "--pool-blocks", "--tile-capacity",
                "--calib-copy-mb", "--no-cpu-baseline"):
        assert opt in r.stdout, opt
