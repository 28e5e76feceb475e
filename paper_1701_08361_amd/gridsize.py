"""Grid-size choice from a measured lookup table (Sec. 3.2, computational cost
reduction; Table oversampling_ratio, Fig. tiny-plot).

The grid side is G = 2 gamma N: the factor 2 is the twofold oversampling that
the convolution with the point-spread function needs, and gamma in [1, 2]
widens the reconstructed field of view to R = G/2 pixels so that an object
larger than the N x N field of view does not alias into it.  The transform
time does not grow smoothly with G, so the method measures every grid size on
the accelerator at hand (once per accelerator generation and transform-library
version), keeps the measurements in a lookup table, and runs each image size N
on the fastest grid with gamma >= 1.4.

Here the table holds, per supported grid side, the device time of one
application of the normal operator DF^H DF (the five fused transform passes of
a CG iteration, nlinv_apply_normal) at batch 1 with J channels, measured with
HIP events.  A table is keyed by the device name, a digest of the kernel
library and J.  The grid sides themselves come from the library: a side is
supported when it accepts a plan for it.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import tempfile
from typing import Dict, List, Optional

GAMMA_MIN = 1.4     # the method's lower bound on gamma
GAMMA_MAX = 2.0     # the upper end of the range gamma may take


def supported_grids(nl, max_side: int = 1024) -> List[int]:
    """Even grid sides up to max_side for which the library has kernels
    (host-only: asks nlinv_sizes, touches no device)."""
    out = []
    for G in range(2, max_side + 1, 2):
        try:
            nl.sizes(nl.make_params(G // 2, 1, 1, G=G))
        except nl.NlinvError:
            continue
        out.append(G)
    return out


def admissible(N: int, grids, gamma_min: float = GAMMA_MIN, gamma_max: float = GAMMA_MAX) -> List[int]:
    """Grid sides G of `grids` with gamma_min <= G / (2N) <= gamma_max, ascending."""
    if N < 1:
        raise ValueError("N must be positive")
    if not (1.0 <= gamma_min <= gamma_max <= 2.0):
        raise ValueError("need 1 <= gamma_min <= gamma_max <= 2")
    return sorted(G for G in grids if gamma_min * 2 * N <= G <= gamma_max * 2 * N)


def choose(N: int, lut: Dict[int, float], gamma_min: float = GAMMA_MIN,
           gamma_max: float = GAMMA_MAX) -> int:
    """The fastest admissible grid side of the table (time per application,
    lower is better); among equal times the smaller grid.  ValueError when the
    table holds no admissible side."""
    cand = admissible(N, lut.keys(), gamma_min, gamma_max)
    if not cand:
        raise ValueError(f"no measured grid side with {gamma_min} <= G/(2*{N}) <= {gamma_max}")
    return min(cand, key=lambda G: (lut[G], G))


def gamma(N: int, G: int) -> float:
    return G / (2.0 * N)


def library_digest(nl) -> str:
    with open(nl.LIB_PATH, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def measure(nl, torch, grids, J: int = 10, K: int = 15, reps: int = 50, warmup: int = 5) -> Dict[int, float]:
    """Microseconds of device time per normal-operator application for every
    grid side in `grids` (batch 1, J channels, a K-spoke radial turn with
    2N samples per spoke, N = G/2).  Random operands; the time does not
    depend on their values."""
    from . import synth
    lut = {}
    for G in grids:
        N = G // 2
        plan = nl.Plan(N, J, K, G=G)
        try:
            traj = torch.from_numpy(synth.radial_trajectory(N, K, 2 * N)).to(plan.device)
            plan.psf(traj, 0)
            gen = torch.Generator(device="cpu").manual_seed(G)
            xh = torch.randn(1, plan.X, dtype=torch.complex64, generator=gen).to(plan.device)
            p = torch.randn(1, plan.X, dtype=torch.complex64, generator=gen).to(plan.device)
            q = plan.empty(1, plan.X)
            for _ in range(warmup):
                plan.apply_normal([0], xh, p, 1.0, q)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                plan.apply_normal([0], xh, p, 1.0, q)
            e1.record()
            e1.synchronize()
            lut[G] = e0.elapsed_time(e1) * 1e3 / reps
        finally:
            plan.close()
    return lut


class GridLUT:
    """Measured tables {G: us}, one per (device, library digest, J), kept in
    memory and, with a path, in a JSON file rewritten atomically on every
    store."""

    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.tables: Dict[str, Dict[int, float]] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if not isinstance(data, dict):
                raise ValueError(f"{path}: not a grid lookup table")
            self.tables = {k: {int(G): float(t) for G, t in v.items()} for k, v in data.items()}

    @staticmethod
    def key(device: str, library: str, J: int) -> str:
        return f"{device}|{library}|J{int(J)}"

    def store(self, key: str, lut: Dict[int, float]):
        for G, t in lut.items():
            if not (t > 0 and math.isfinite(t)):
                raise ValueError(f"time of grid {G} must be positive and finite, got {t}")
        self.tables[key] = {int(G): float(t) for G, t in lut.items()}
        if self.path:
            d = os.path.dirname(os.path.abspath(self.path))
            fd, tmp = tempfile.mkstemp(dir=d, prefix=".grid-", suffix=".json")
            with os.fdopen(fd, "w") as f:
                json.dump({k: {str(G): t for G, t in v.items()} for k, v in self.tables.items()}, f, indent=1)
            os.replace(tmp, self.path)

    def get(self, key: str) -> Optional[Dict[int, float]]:
        return self.tables.get(key)

    def table(self, nl, torch, J: int = 10, K: int = 15, grids=None, reps: int = 50) -> Dict[int, float]:
        """The table of the current device, library and J, measured and stored
        when absent."""
        key = self.key(torch.cuda.get_device_name(), library_digest(nl), J)
        lut = self.get(key)
        if lut is None:
            lut = measure(nl, torch, grids if grids is not None else supported_grids(nl), J=J, K=K, reps=reps)
            self.store(key, lut)
        return lut
