"""The benchmark script's argument contract, on the CPU: more than one GPU is refused with a
message and exit status 2 (the library runs on one GPU), and an unknown leg is an argument error;
neither touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_leg_is_an_argument_error():
    r = run("--legs", "headline,bogus")
    assert r.returncode == 2
    assert "unknown legs" in r.stderr and r.stdout == ""
