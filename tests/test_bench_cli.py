"""The benchmark's command-line contract that holds without a GPU: more than one GPU is
refused with a message and a non-zero status before any device is touched, and the options
parse.  Also the source hash that ties the measured constants to the code they were measured
on: it ignores comments, follows every code change, and matches the committed sources."""
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


def test_source_hash_ignores_comments_but_not_code(tmp_path):
    # the measured constants (rocprofv3 traffic, VALU and fp64 counts) are tied to the code
    # by a hash of the sources without comments: comment and blank-space edits keep it, any
    # change to the code, or to a string literal that looks like a comment, does not
    import bench

    src = 'int f(int x) { // the "quoted" part\n  return x /* two */ + 2; }\nconst char *s = "a // b";\n'
    same = '// a header\nint f(int x) {\n\n  return x  + 2;   // changed comment\n}\nconst char *s = "a // b";\n'
    code = 'int f(int x) { // the "quoted" part\n  return x /* two */ + 3; }\nconst char *s = "a // b";\n'
    lit = 'int f(int x) { // the "quoted" part\n  return x /* two */ + 2; }\nconst char *s = "a // c";\n'
    texts = {}
    for name, t in (("src", src), ("same", same), ("code", code), ("lit", lit)):
        p = tmp_path / f"{name}.hpp"
        p.write_text(t)
        texts[name] = bench._code_text(str(p))
    assert texts["src"] == texts["same"]
    assert texts["src"] != texts["code"]
    assert texts["src"] != texts["lit"]
    assert '"a // b"' in texts["src"] and "/*" not in texts["src"]
    # the hashes the bench's constants carry are those of the sources as they are
    assert bench.kernel_src_hash() == bench.MEASURED_TRAFFIC["src_hash"]
    assert bench.angle_step_src_hash() == bench.ANGLE_STEP_COUNTERS["src_hash"]
    assert bench.angle_src_hash(3) == bench.ANGLE_COUNTERS[3]["src_hash"]
    assert bench.angle_src_hash(2) == bench.ANGLE_COUNTERS[2]["src_hash"]
