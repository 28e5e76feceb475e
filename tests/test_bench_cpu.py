"""Host-side checks of bench.py that need no GPU: the one-GPU refusal and the
kernel-source hash that keys the committed counter summary."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_source_hash_and_counter_summary_format():
    r = _run("--source-hash")
    assert r.returncode == 0
    h = r.stdout.strip()
    assert len(h) == 16 and int(h, 16) >= 0
    with open(os.path.join(ROOT, "profiles", "nlinv_toeplitz_rows_series160_pmc.md")) as f:
        lines = [l.split() for l in f if l.startswith("kernel_sources:") or l.startswith("traffic:")]
    assert lines and lines[0][0] == "kernel_sources:" and len(lines[0][1]) == 16
    assert all(t[0] == "traffic:" and t[1] == "toeplitz_rows" and int(t[4]) > 0 for t in lines[1:])
