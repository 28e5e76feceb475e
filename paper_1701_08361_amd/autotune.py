"""Autotuning of the parallelisation parameters (Sec. 3.3, autotuning).

The method records the run time of every reconstruction together with its
acquisition and reconstruction parameters and its parallelisation setting in
a database, (protocol) -> (setting) -> frames/s.  For a protocol it picks the
setting with the best recorded rate; a learning mode instead picks settings
not yet recorded for the protocol, so that a setup phase can fill the
database; a protocol never seen before gets the best setting of the nearest
recorded protocol.

The paper's setting is (T, A): T reconstruction threads working on frames
concurrently (temporal decomposition) and A accelerators per thread (channel
decomposition).  On one GPU the setting is
  T      frames reconstructed together in one relaxed group of the equation
         for h(n, m) after l = U strict frames (T = 1 is the strict order,
         all T give the method's images: the paper's prerequisite that every
         setting yields the same image quality);
  A      accelerators per frame, 1 here (no channel decomposition);
  graphs HIP-graph replay of the launch sequences: a capture costs time once
         per distinct argument set, a replay saves the per-kernel launch cost
         of every later frame, so the better choice depends on the number of
         frames.
The search space for A = 1 is T = 1..8, as in the paper, times graphs off/on.
A tuner may also search the tile schedule of the CG column passes
(col_tile: columns per block, 8 or 4; the same images bit for bit) and the
pass fusion of a CG iteration (cg_passes: six dependent kernels, or four with
the direction update, the coil rows of the direction and the vector step
folded into the operator's passes; the same images to rounding) and the
factorisation G = G1 G2 of the Toeplitz row pass's transforms (fft_split: the
grid's default or its alternative; the same images to rounding), so that the
kernel decomposition is measured per protocol instead of fixed.

The database is a JSON file (a list of records); the runner reconstructs a
whole series through the C-ABI and measures it with the host clock around
synchronised GPU work.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

PROTOCOL_KEYS = ("mode", "N", "J", "K", "U", "frames", "newton", "cg")


def _norm_protocol(p: Dict) -> Dict:
    missing = [k for k in PROTOCOL_KEYS if k not in p]
    if missing:
        raise ValueError(f"protocol lacks {missing}")
    return {k: p[k] for k in PROTOCOL_KEYS}


def search_space(gpus: int = 1, max_T: int = 8, tiles: Optional[Sequence[int]] = None,
                 passes: Optional[Sequence[int]] = None, splits: Optional[Sequence[int]] = None) -> List[Dict]:
    """Settings (T, A, graphs): for A = 1, T = 1..max_T; for A = 2 up to
    max_T / 2; for A = 3, 4 up to max_T / 4 (the paper's limits on 8 GPUs),
    with A <= gpus; each with graphs off and on; with `tiles`, each also with
    every listed column-pass tile schedule (col_tile); with `passes`, each
    also with every listed CG pass fusion (cg_passes, 4 or 6); with `splits`,
    each also with every listed Toeplitz-pass factorisation (fft_split, 0 or 1)."""
    if tiles is not None and (not tiles or any(t not in (4, 8) for t in tiles)):
        raise ValueError("tile schedules are 4 or 8 columns per block")
    if passes is not None and (not passes or any(p not in (4, 6) for p in passes)):
        raise ValueError("a CG iteration has 4 or 6 passes")
    if splits is not None and (not splits or any(f not in (0, 1) for f in splits)):
        raise ValueError("factorisations are 0 (the grid's default) and 1 (its alternative)")
    out = []
    for A in (1, 2, 3, 4):
        if A > gpus:
            break
        tmax = max_T if A == 1 else (max_T // 2 if A == 2 else max(1, max_T // 4))
        for T in range(1, tmax + 1):
            for graphs in (False, True):
                base = [{"T": T, "A": A, "graphs": graphs}]
                if tiles is not None:
                    base = [dict(c, col_tile=int(t)) for c in base for t in tiles]
                if passes is not None:
                    base = [dict(c, cg_passes=int(p)) for c in base for p in passes]
                if splits is not None:
                    base = [dict(c, fft_split=int(f)) for c in base for f in splits]
                out.extend(base)
    return out


class TuningDB:
    """(protocol, setting, frames/s) records, kept in memory and, with a path,
    in a JSON file rewritten atomically after every insert."""

    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.records: List[Dict] = []
        if path and os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if not isinstance(data, list):
                raise ValueError(f"{path}: not a tuning database")
            self.records = [r for r in data if {"protocol", "config", "fps"} <= set(r)]

    def insert(self, protocol: Dict, config: Dict, fps: float):
        if not (fps > 0 and math.isfinite(fps)):
            raise ValueError(f"run rate must be positive and finite, got {fps}")
        self.records.append({"protocol": _norm_protocol(protocol), "config": dict(config), "fps": float(fps)})
        self.save()

    def save(self):
        if not self.path:
            return
        d = os.path.dirname(os.path.abspath(self.path))
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune-", suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump(self.records, f, indent=1)
        os.replace(tmp, self.path)

    def lookup(self, protocol: Dict) -> List[Tuple[Dict, float]]:
        """Recorded (setting, frames/s) of a protocol, fastest first."""
        p = _norm_protocol(protocol)
        hits = [(r["config"], r["fps"]) for r in self.records if r["protocol"] == p]
        return sorted(hits, key=lambda cf: -cf[1])

    def protocols(self) -> List[Dict]:
        seen = []
        for r in self.records:
            if r["protocol"] not in seen:
                seen.append(r["protocol"])
        return seen


def protocol_distance(a: Dict, b: Dict) -> float:
    """Order of similarity between protocols: another imaging mode is
    infinitely far; otherwise the sum of |log| ratios of the sizes, the frame
    count, the channels and the iteration counts (data size first: N and K
    count twice)."""
    if a["mode"] != b["mode"]:
        return math.inf
    lr = lambda k: abs(math.log(max(a[k], 1) / max(b[k], 1)))
    return 2 * lr("N") + 2 * lr("K") + lr("frames") + lr("J") + lr("U") + lr("newton") + lr("cg")


class Autotuner:
    def __init__(self, db: TuningDB, gpus: int = 1, max_T: int = 8, learning: bool = False,
                 tiles: Optional[Sequence[int]] = None, passes: Optional[Sequence[int]] = None,
                 splits: Optional[Sequence[int]] = None):
        self.db, self.learning = db, learning
        self.space = search_space(gpus, max_T, tiles, passes, splits)

    def untried(self, protocol: Dict) -> List[Dict]:
        tried = [c for c, _ in self.db.lookup(protocol)]
        return [c for c in self.space if c not in tried]

    def choose(self, protocol: Dict) -> Dict:
        """Learning mode: the first setting without a record for this protocol.
        Otherwise the fastest recorded setting; for an unseen protocol the
        fastest setting of the nearest recorded one; with no records at all,
        the strict order with graphs."""
        if self.learning:
            todo = self.untried(protocol)
            if todo:
                return todo[0]
        hits = self.db.lookup(protocol)
        if hits:
            return hits[0][0]
        p = _norm_protocol(protocol)
        near = sorted(((protocol_distance(p, q), i, q) for i, q in enumerate(self.db.protocols())),
                      key=lambda t: (t[0], t[1]))
        for d, _, q in near:
            if math.isfinite(d):
                return self.db.lookup(q)[0][0]
        return {"T": 1, "A": 1, "graphs": True}

    def record(self, protocol: Dict, config: Dict, fps: float):
        self.db.insert(protocol, config, fps)

    def learn(self, protocol: Dict, run: Callable[[Dict], float]) -> Dict:
        """Measure every untried setting of the protocol (run(config) ->
        frames/s), record each, and return the fastest setting."""
        for c in self.untried(protocol):
            self.record(protocol, c, run(c))
        return self.db.lookup(protocol)[0][0]


def run_series(nl, torch, traj, y, turns, config: Dict, newton: int, cg: int, U: int,
               l: Optional[int] = None) -> Tuple[float, object]:
    """Reconstruct a whole series under `config` and return (frames/s, image of
    the last frame).  traj [F][K][S_r][2], y [F][J][S] device tensors, turns
    the F turn indices.  Frames 0..l (default l = U) run strictly, the rest in
    groups of config["T"] (the last group may be shorter).  The plan and the
    PSF kernels of the U turns are built before the clock starts; gridding,
    reconstruction and graph captures are timed."""
    if config.get("A", 1) != 1:
        raise ValueError("one GPU: A must be 1")
    T = int(config["T"])
    F, J = y.shape[0], y.shape[1]
    N = int(round(traj.shape[2] / 2))
    K = traj.shape[1]
    l = U if l is None else l
    plan = nl.Plan(N, J, K, U=U, batch=T, newton=newton, cg=cg, col_tile=int(config.get("col_tile", 0)),
                   cg_passes=int(config.get("cg_passes", 0)), fft_split=int(config.get("fft_split", 0)))
    try:
        plan.set_graphs(bool(config.get("graphs", True)))
        for t in range(min(U, F)):
            plan.psf(traj[t].contiguous(), int(turns[t]))
        dev = y.device
        z = torch.empty(T, J, plan.R, plan.R, dtype=torch.complex64, device=dev)
        xb = [torch.empty(T, plan.X, dtype=torch.complex64, device=dev) for _ in range(2)]
        img = torch.empty(T, plan.R, plan.R, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev, par, n = None, 0, 0
        while n < F:
            k = 1 if n <= l else min(T, F - n)
            plan.set_batch(k)
            ts = [int(t) for t in turns[n:n + k]]
            plan.grid(traj[n:n + k], y[n:n + k], turns=ts, z=z[:k])
            plan.set_batch(T)
            out = xb[par][:k]
            plan.reconstruct_frames(z[:k], ts, xprev=prev, xhat=out, img=img[:k])
            prev = xb[par][k - 1]
            last = img[k - 1]
            par ^= 1
            n += k
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return F / dt, last.clone()
    finally:
        plan.close()
