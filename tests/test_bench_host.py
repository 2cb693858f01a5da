"""Host-side behaviour of bench.py that needs no GPU: the one-GPU contract and the
kernel-source digest that guards the committed counter figures."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_digest_is_a_sha256_of_the_solver_sources():
    r = _run("--kernel-digest")
    assert r.returncode == 0
    digest = r.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{64}", digest)
    # counter files carry a digest of the same form; bench.py uses their figures only on a match
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.endswith("_counters.md"):
            text = open(os.path.join(ROOT, "profiles", name)).read()
            m = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
            assert m and len(m.group(1)) == 64, name
