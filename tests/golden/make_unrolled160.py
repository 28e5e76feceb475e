"""Writes unrolled160.json: the FP64 oracle's IRGNM (Sec. 2.2) on one frame
of the 160 px, 10-coil, 15-spoke real-time series (5 Newton steps of 20 CG
iterations, alpha_0 = 1, Sobolev weight (880, 16)), the loss
L = ||image - phantom||^2 on the combined image |rho| sqrt(sum_j |c_j|^2),
sampled image pixels, and the derivatives of L along eight seeded data
directions and in alpha_0, a and l, each by central differences of the
oracle's reconstruction at two steps h and h/2, combined by Richardson
extrapolation (the file also keeps both estimates and their relative spread).  It calls only the oracle and the
seeded input generators.  Takes about half an hour on 8 cores (45 oracle reconstructions):

    python tests/golden/make_unrolled160.py
"""
from __future__ import annotations

import json
import os
import sys
from multiprocessing import Pool

os.environ.setdefault("OMP_NUM_THREADS", "1")       # one BLAS thread per worker process
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import nlinv_oracle as O  # noqa: E402
from paper_1701_08361_amd import synth  # noqa: E402

CASE = dict(seed=73, N=160, J=10, K=15, newton=5, cg=20, alpha0=1.0, a=880.0, l=16.0)
DIRECTIONS = list(range(1601, 1609))   # seeds of the data directions u_k (synth.random_samples)
REL_STEP = {"alpha0": 1e-4, "a": 1e-4, "l": 1e-5, "y": 1e-4}
N_PIXELS = 64


def _series():
    c = CASE
    return synth.real_time_series(seed=c["seed"], N=c["N"], J=c["J"], J_phys=30, K=c["K"], U=1, frames=1)


def _image(shift):
    """The oracle's image with (alpha0, a, l) moved by `shift` and the data
    moved by t u along direction seed k: shift = {"alpha0": d, ...,
    "y": (seed, t)}."""
    c = CASE
    s = _series()
    y = s.y[0].astype(np.complex128)
    if "y" in shift:
        seed, t = shift["y"]
        y = y + t * synth.random_samples(seed, c["J"], y.shape[-1]).astype(np.complex128)
    g = O.Geometry.make(c["N"], c["J"], a=c["a"] + shift.get("a", 0.0), l=c["l"] + shift.get("l", 0.0))
    traj = s.traj[0].astype(np.float64)
    x = O.reconstruct(g, O.grid(y, traj, g.R), O.psf_kernel(traj, g.R, g.G), newton=c["newton"],
                      cg_iters=c["cg"], alpha0=c["alpha0"] + shift.get("alpha0", 0.0))
    return O.image(g, x)


def main():
    c = CASE
    s = _series()
    truth = s.truth[0] * np.linalg.norm(s.coils.reshape(c["J"], -1), axis=0).reshape(c["N"], c["N"])
    ynorm = float(np.linalg.norm(s.y[0].astype(np.complex128)))
    steps = {}
    for k in ("alpha0", "a", "l"):
        steps[k] = REL_STEP[k] * c[k]
    for i, seed in enumerate(DIRECTIONS):
        u = synth.random_samples(seed, c["J"], s.y.shape[-1]).astype(np.complex128)
        steps[f"y.u{i}"] = REL_STEP["y"] * ynorm / float(np.linalg.norm(u))
    jobs = [{}]
    for k, h in steps.items():
        for frac in (1.0, 0.5):
            for sign in (1.0, -1.0):
                d = sign * frac * h
                if k.startswith("y."):
                    jobs.append({"y": (DIRECTIONS[int(k[3:])], d)})
                else:
                    jobs.append({k: d})
    with Pool(min(8, len(jobs))) as pool:
        imgs = pool.map(_image, jobs)
    base = imgs[0]
    scale = float(np.linalg.norm(base) / np.linalg.norm(truth))
    target = truth * scale

    def loss(img):
        return float(np.sum((img - target) ** 2))

    deriv, spread, raw = {}, {}, {}
    it = iter(imgs[1:])
    for k, h in steps.items():
        lp, lm, lp2, lm2 = (loss(next(it)) for _ in range(4))
        d1 = (lp - lm) / (2 * h)
        d2 = (lp2 - lm2) / h
        deriv[k] = d2 + (d2 - d1) / 3          # Richardson: the h^2 terms cancel
        spread[k] = abs(d1 - d2) / abs(d2)
        raw[k] = [d1, d2]
    rng = np.random.default_rng(160)
    idx = np.sort(rng.choice(base.size, N_PIXELS, replace=False))
    out = {
        "what": "FP64 oracle IRGNM on frame 0 of the 160 px real-time series; loss ||image - s * phantom||^2 "
                "(s = truth_scale); derivatives by central differences of the oracle at steps h and h/2, "
                "Richardson-extrapolated (both estimates in fd_h_and_half_h, their relative spread in "
                "fd_spread); data directions "
                "u_k = synth.random_samples(seed_k, J, S)",
        "case": dict(c, truth_scale=scale),
        "data_directions": [{"seed": sd} for sd in DIRECTIONS],
        "steps": steps,
        "loss": loss(base),
        "image_norm": float(np.linalg.norm(base)),
        "pixels": {"index": idx.tolist(), "value": base.ravel()[idx].tolist()},
        "derivatives": deriv,
        "fd_spread": spread,
        "fd_h_and_half_h": raw,
    }
    with open(os.path.join(HERE, "unrolled160.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"loss": out["loss"], "derivatives": deriv, "fd_spread": spread}, indent=1))


if __name__ == "__main__":
    main()
