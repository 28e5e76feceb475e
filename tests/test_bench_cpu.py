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


def test_roofline_fraction_per_batch_on_complex64_bytes():
    """The roofline object on synthetic launch times: per batch size B, frac is
    (B J G R 16 + G^2 4) bytes (the grid rows in and out at complex64 size,
    one PSF kernel) over the average launch duration, against 8 TB/s; batch
    sizes are listed apart, never blended, and the headline is the asked one."""
    sys.path.insert(0, ROOT)
    import bench
    N, J = bench.N, bench.J
    G, R = 2 * N, N
    kt = {1: {"toeplitz_rows": (0.010 * 100, 100)},      # 10 us per launch
          16: {"toeplitz_rows": (0.050 * 40, 40)}}       # 50 us per launch
    rl = bench.roofline(kt, 16)
    assert rl["batch"] == 16 and rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    for B, t in ((1, 10e-6), (16, 50e-6)):
        alg = B * J * G * R * 16 + G * G * 4
        by = rl["by_batch"][str(B)]
        assert abs(by["algorithmic_bytes"] - alg) < 1e-6 * alg
        assert abs(by["frac"] - alg / t / 8e12) < 1e-9
        assert abs(by["storage_gbs"] - (B * J * G * R * 32 + G * G * 4) / t / 1e9) < 1e-6
    assert rl["frac"] == rl["by_batch"]["16"]["frac"]
    assert bench.roofline({1: {"toeplitz_rows": (0.01, 1)}}, 16) is None
