"""The benchmark's command-line contract that holds without a GPU: more than one GPU is
refused with a message and a non-zero status before any device is touched, and the options
parse."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "4", "--steps", "1")
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 4 and "one GPU" in out["error"]


def test_options_parse():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--gpus", "--eps-cut", "--autotune", "--batch", "--serve", "--first-passage",
                "--pair-probs", "--scale", "--workload", "--precision"):
        assert opt in r.stdout, opt
