"""Benchmark of the NLINV hot path on one MI355X.

Workload: the real-time series of 160 px frames (320 x 320 grid), 10 virtual
coils (PCA from 30), 15 spokes x 320 samples per frame in 5 rotated turns,
7 Newton x 20 CG steps, temporal regularisation to the previous frame.
A step is one frame per series: gridding (z = F^H y by Kaiser-Bessel gridding
through the turn's table; the PSF kernel and the table of each turn are built
once at set-up) and the IRGNM reconstruction.

  plain   : one series, frames solved one after another (batch 1)  -> `value`
  batched : 16 independent series advanced together (batch 16)    -> `batched`

Inputs are seeded synthetic data generated on the host before timing and
copied to the GPU; the timed region starts with everything resident in HBM.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, J, J_PHYS, K, U, M, C = 160, 10, 30, 15, 5, 7, 20
HBM_PEAK_GBS = 8000.0

# rocprofv3 HBM counter summary of the roofline kernel (FETCH_SIZE / WRITE_SIZE
# per dispatch, scaled by a plain copy of known size), and the sources it was
# taken on: the figures are used only while those sources are unchanged.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "nlinv_toeplitz_rows_series160_pmc.md")
KERNEL_SOURCES = ["paper_1701_08361_amd/csrc/nlinv_fft.h", "paper_1701_08361_amd/csrc/nlinv_kernels.h",
                  "paper_1701_08361_amd/csrc/nlinv_internal.h"]


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace collapsed, so that the
    hash follows the code the counters measured and not its comments."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kind: str):
    """{batch: HBM bytes per launch} of kernel class `kind` from the counter
    summary, or None if there is none for the current kernel sources."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    src, out = None, {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            t = line.split()
            if len(t) == 2 and t[0] == "kernel_sources:":
                src = t[1]
            elif len(t) == 5 and t[0] == "traffic:" and t[1] == kind and t[2] == "batch":
                out[int(t[3])] = float(t[4])
    if src != kernel_source_hash() or not out:
        return None
    return out


COL_TILE = 0   # tile schedule of the plain, relaxed and batched plans (--col-tile)

# Mixed sizes: (N, J, K, series) per shape, 16 series in all
MIXED = [(128, 8, 11, 5), (160, 10, 15, 6), (192, 16, 21, 5)]
# Streaming slices: (N, J virtual, J_phys receive channels, K)
SLICES = [(128, 8, 20, 9), (160, 10, 32, 15), (192, 12, 48, 17), (224, 16, 64, 21)]


def _raw_series(args):
    seed, frames, n, j, jp, k = args
    from threadpoolctl import threadpool_limits
    from paper_1701_08361_amd import synth
    with threadpool_limits(1):
        s = synth.real_time_series(seed=seed, N=n, J=j, J_phys=jp, K=k, U=U, frames=frames, compress=False)
    return s.traj, s.y, s.turn


def _series(args):
    seed, frames, threads = args[:3]
    n, j, k = args[3:] if len(args) > 3 else (N, J, K)
    from threadpoolctl import threadpool_limits
    from paper_1701_08361_amd import synth
    with threadpool_limits(threads):
        s = synth.real_time_series(seed=seed, N=n, J=j, J_phys=max(J_PHYS, 2 * j), K=k, U=U, frames=frames)
    # the phantom's combined image of frame 0 (target of the differentiation run)
    target = s.truth[0] * np.linalg.norm(s.coils.reshape(j, -1), axis=0).reshape(n, n) * s.scale
    return s.traj, s.y, s.turn, target


def pool_map(fn, jobs, workers):
    """fn over jobs in a fork pool that is closed and joined (the workers exit
    on their own instead of being terminated)."""
    if workers <= 1 or len(jobs) <= 1:
        return [fn(a) for a in jobs]
    pool = mp.get_context("fork").Pool(min(workers, len(jobs)))
    try:
        out = pool.map(fn, jobs)
    finally:
        pool.close()
        pool.join()
    return out


def make_data(seeds, frames, workers):
    if workers > 1 and len(seeds) > 1:
        return pool_map(_series, [(s, frames, 1) for s in seeds], workers)
    return [_series((s, frames, None)) for s in seeds]


def kernel_bytes(kind: str, B: int, turns_distinct: int = 1, grid_bytes: int = 8) -> float:
    """Algorithmic HBM bytes of one launch of a kernel class: each input read
    once, each output written once, every complex array at complex64 size
    (8 B), the half-transformed grid at `grid_bytes` per value (8: complex64,
    the algorithmic size; 16: the float64 storage of the last Newton step)."""
    G, R, Gc = 2 * N, N, N // 2
    s2 = grid_bytes
    if kind in ("toeplitz_rows", "toeplitz_rows_f64"):   # grid rows in + out, PSF kernel rows
        return B * J * G * R * 2 * s2 + turns_distinct * G * G * 4
    if kind == "coil_cols":          # coil rows in, coil images + image + direction in, grid out
        return B * J * (Gc * R * 8 + R * R * 8 + G * R * s2) + B * R * R * (8 + 8 + 8)
    if kind == "back_cols":          # grid in, coils in, PR out, coil rows out
        return B * J * (G * R * s2 + R * R * 8 + R * R * 8 + Gc * R * 8) + B * R * R * (8 + 8)
    raise ValueError(kind)


def compulsory_bytes_per_cg() -> float:
    """Compulsory bytes of one CG iteration of one item (complex64): read the
    direction, the coil images, the image, the PSF kernel and the Sobolev
    weights, write the operator output."""
    G, R, Gc = 2 * N, N, N // 2
    X = R * R + J * Gc * Gc
    return X * 8 + J * R * R * 8 + R * R * 8 + G * G * 4 + Gc * Gc * 4 + X * 8


def run_mode(torch, nl, data, B, steps, warmup, timer_kernels, kt_frames, graphs, img_store=None, flags=0,
             cg_passes=0, fft_split=0):
    """Advance B series by warmup + steps frames (timed), then kt_frames more
    per kernel class in `timer_kernels` with the class's launches timed by HIP
    events.  Returns per-step ms, total ms of the timed steps, and
    {class: (ms, launches)}.  img_store[n] (optional) receives the image of
    frame n of item 0."""
    plan = nl.Plan(N, J, K, U=U, batch=B, newton=M, cg=C, flags=flags, col_tile=COL_TILE, cg_passes=cg_passes,
                   fft_split=fft_split)
    plan.set_graphs(graphs)
    import numpy as np
    traj = torch.from_numpy(np.stack([d[0] for d in data], axis=1)).cuda()  # [F,B,K,S_r,2]
    y = torch.from_numpy(np.stack([d[1] for d in data], axis=1)).cuda()     # [F,B,J,S]
    turn = data[0][2]
    F = traj.shape[0]
    z = torch.empty(B, J, N, N, dtype=torch.complex64, device="cuda")
    xa = torch.empty(B, plan.X, dtype=torch.complex64, device="cuda")
    xb = torch.empty_like(xa)
    img = torch.empty(B, N, N, dtype=torch.float32, device="cuda")
    # every PSF kernel is computed once up front (part of plan set-up, not of a frame)
    for t in range(U):
        plan.psf(traj[t, 0].contiguous(), t)
    torch.cuda.synchronize()

    def frame(n, xprev, xout):
        f = n % F
        tn = [int(turn[f])] * B
        plan.grid(traj[f], y[f], turns=tn, z=z)
        plan.reconstruct(z, tn, xprev=xprev, xhat=xout, init=(1 if xprev is None else 2), img=img)
        if img_store is not None and n < img_store.shape[0]:
            img_store[n].copy_(img[0])

    xprev = None
    bufs = [xa, xb]
    # with HIP graphs, every (turn, buffer parity) argument set is captured
    # before the clock starts, whatever the warm-up count: frame 0 starts from
    # the unit point, frames 1 .. 2U see every set of the regularised frames
    nwarm = max(warmup, 2 * U + 1) if graphs else warmup
    for n in range(nwarm):
        frame(n, xprev, bufs[n & 1])
        xprev = bufs[n & 1]
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        n = nwarm + i
        ev[i][0].record()
        frame(n, xprev, bufs[n & 1])
        ev[i][1].record()
        xprev = bufs[n & 1]
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    per = [a.elapsed_time(b) for a, b in ev]
    kt = {}
    n = nwarm + steps
    for kernel in (timer_kernels if kt_frames > 0 else []):
        # per-kernel HIP events need uncaptured launches; same kernels, same sizes
        plan.timer_enable(kernel)
        for i in range(kt_frames):
            frame(n, xprev, bufs[n & 1])
            xprev = bufs[n & 1]
            n += 1
        kt[kernel] = plan.timer_read()
        plan.timer_enable("none")
    plan.close()
    return per, total_ms, kt


def run_split(torch, nl, data, B, P, steps, warmup, cg_passes=0, fft_split=0):
    """B series advanced together as P plans of B / P series each, every step
    one HIP graph launch of all P reconstructions (nlinv_reconstruct_multi,
    one branch per plan, after each plan's gridding on the same stream): the
    plans' kernels overlap, so one plan's kernel boundaries and tails are
    hidden behind the other's work.  Each item reconstructs the same bits as
    in one plan of batch B.  Returns per-step ms and total ms."""
    import numpy as np
    assert B % P == 0
    b = B // P
    runs = []
    for k in range(P):
        part = data[k * b:(k + 1) * b]
        plan = nl.Plan(N, J, K, U=U, batch=b, newton=M, cg=C, col_tile=COL_TILE, cg_passes=cg_passes,
                       fft_split=fft_split)
        traj = torch.from_numpy(np.stack([d[0] for d in part], axis=1)).cuda()   # [F,b,K,S_r,2]
        y = torch.from_numpy(np.stack([d[1] for d in part], axis=1)).cuda()      # [F,b,J,S]
        for t in range(U):
            plan.psf(traj[t, 0].contiguous(), t)
        z = torch.empty(b, J, N, N, dtype=torch.complex64, device="cuda")
        xs = [torch.empty(b, plan.X, dtype=torch.complex64, device="cuda") for _ in range(2)]
        img = torch.empty(b, N, N, dtype=torch.float32, device="cuda")
        runs.append(dict(plan=plan, traj=traj, y=y, z=z, xs=xs, img=img))
    turn = data[0][2]
    F = runs[0]["traj"].shape[0]
    torch.cuda.synchronize()

    def frame(n):
        f = n % F
        tn = [int(turn[f])] * b
        for r in runs:
            r["plan"].grid(r["traj"][f], r["y"][f], turns=tn, z=r["z"])
        nl.reconstruct_multi([r["plan"] for r in runs], [r["z"] for r in runs], [tn] * P,
                             xprevs=[None if n == 0 else r["xs"][(n - 1) & 1] for r in runs],
                             xhats=[r["xs"][n & 1] for r in runs], inits=[1 if n == 0 else 2] * P,
                             imgs=[r["img"] for r in runs])

    # every (turn, buffer parity) graph is captured before the clock
    nwarm = max(warmup, 2 * U + 1)
    for n in range(nwarm):
        frame(n)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        frame(nwarm + i)
        ev[i][1].record()
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    per = [a.elapsed_time(e) for a, e in ev]
    for r in runs:
        r["plan"].close()
    return per, total_ms


def run_relaxed(torch, nl, data, steps, warmup, l, o, graphs, img_store=None, cg_passes=0):
    """One series under the relaxed temporal coupling: frames 0..l in strict
    order, then groups of o frames (nlinv_reconstruct_frames).  Times the
    groups that start at or after frame `warmup`, about `steps` frames.
    Returns (frames timed, total ms, per-group ms, frames processed)."""
    plan = nl.Plan(N, J, K, U=U, batch=o, newton=M, cg=C, col_tile=COL_TILE, cg_passes=cg_passes)
    plan.set_graphs(graphs)
    traj = torch.from_numpy(data[0][0]).cuda()      # [F, K, S_r, 2]
    y = torch.from_numpy(data[0][1]).cuda()         # [F, J, S]
    turn = data[0][2]
    F = traj.shape[0]
    for t in range(U):
        plan.psf(traj[t].contiguous(), t)
    z = torch.empty(o, J, N, N, dtype=torch.complex64, device="cuda")
    xb = [torch.empty(o, plan.X, dtype=torch.complex64, device="cuda") for _ in range(2)]
    img = torch.empty(o, N, N, dtype=torch.float32, device="cuda")
    zs = {k: z[:k] for k in range(1, o + 1)}
    imgs = {k: img[:k] for k in range(1, o + 1)}
    torch.cuda.synchronize()
    state = {"prev": None, "par": 0}

    def group(n, k):
        fs = [(n + i) % F for i in range(k)]
        plan.set_batch(k)
        if fs == list(range(fs[0], fs[0] + k)):
            plan.grid(traj[fs[0]:fs[0] + k], y[fs[0]:fs[0] + k], turns=[int(turn[f]) for f in fs], z=zs[k])
        else:
            plan.grid(traj[fs].contiguous(), y[fs].contiguous(), turns=[int(turn[f]) for f in fs], z=zs[k])
        plan.set_batch(o)
        out = xb[state["par"]][:k]
        plan.reconstruct_frames(zs[k], [int(turn[f]) for f in fs], xprev=state["prev"], xhat=out, img=imgs[k])
        state["prev"] = xb[state["par"]][k - 1]
        state["par"] ^= 1
        if img_store is not None:
            for i in range(k):
                if n + i < img_store.shape[0]:
                    img_store[n + i].copy_(img[i])

    n = 0
    while n <= l:                      # strict frames
        group(n, 1)
        n += 1
    # untimed groups until every (turn phase, buffer parity) graph has been captured
    while n < max(warmup, l + 1 + 2 * U * o):
        group(n, o)
        n += o
    torch.cuda.synchronize()
    ngroups = max(1, steps // o)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(ngroups)]
    t0 = time.perf_counter()
    for g in range(ngroups):
        ev[g][0].record()
        group(n, o)
        ev[g][1].record()
        n += o
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    plan.close()
    return ngroups * o, total, [a.elapsed_time(b) for a, b in ev], n


def run_serving(torch, nl, data, S, periods, period_ms, policy, graphs, cg_passes=0):
    """S slices streamed at 1000 / period_ms frames/s each; the S frames of
    period k arrive together at k * period_ms (after 2U untimed warm-up
    periods that capture the graphs).
      plain   : every frame is solved alone (batch 1) as soon as it arrives,
                first come first served on one stream;
      batched : when the GPU is free, the oldest pending period's frames
                (one per slice) are solved as one batch of S.
    Latency = completion (HIP event) - arrival.  Returns (latencies ms,
    frames, wall ms)."""
    B = 1 if policy == "plain" else S
    plan = nl.Plan(N, J, K, U=U, batch=B, newton=M, cg=C, cg_passes=cg_passes)
    plan.set_graphs(graphs)
    traj = torch.from_numpy(np.stack([d[0] for d in data[:S]], axis=1)).cuda()  # [F,S,K,S_r,2]
    y = torch.from_numpy(np.stack([d[1] for d in data[:S]], axis=1)).cuda()     # [F,S,J,S]
    turn = data[0][2]
    F = traj.shape[0]
    for t in range(U):
        plan.psf(traj[t, 0].contiguous(), t)
    X = plan.X
    state = torch.empty(2, S, X, dtype=torch.complex64, device="cuda")   # ping-pong per period
    z = torch.empty(B, J, N, N, dtype=torch.complex64, device="cuda")
    img = torch.empty(B, N, N, dtype=torch.float32, device="cuda")

    def solve_period(k):
        f = k % F
        tn = int(turn[f])
        cur, prev = state[k & 1], state[(k - 1) & 1]
        if policy == "plain":
            for s in range(S):
                plan.grid(traj[f, s:s + 1], y[f, s:s + 1], turns=[tn], z=z)
                plan.reconstruct(z, [tn], xprev=None if k == 0 else prev[s:s + 1], xhat=cur[s:s + 1],
                                 init=1 if k == 0 else 2, img=img)
                yield s
        else:
            plan.grid(traj[f], y[f], turns=[tn] * S, z=z)
            plan.reconstruct(z, [tn] * S, xprev=None if k == 0 else prev, xhat=cur,
                             init=1 if k == 0 else 2, img=img)
            yield S - 1

    warm = 2 * U
    for k in range(warm):
        for _ in solve_period(k):
            pass
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    done = []                          # (event, arrival ms)
    t0 = time.perf_counter()
    start.record()
    last = None
    for i in range(periods):
        k = warm + i
        arrival = i * period_ms
        now = (time.perf_counter() - t0) * 1e3
        if now < arrival:
            time.sleep((arrival - now) / 1e3)
        if policy == "batched" and last is not None:
            last.synchronize()           # the GPU takes the next batch when it is free
        for s in solve_period(k):
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            n_done = 1 if policy == "plain" else S
            done.append((ev, arrival, n_done))
            last = ev
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    lat = []
    for ev, arrival, n in done:
        lat += [start.elapsed_time(ev) - arrival] * n
    plan.close()
    return lat, S * periods, wall


def run_mixed(torch, nl, groups, steps, warmup, concurrent, graphs, one_graph=False):
    """Series of several shapes advanced together, one batched plan per shape:
    one after another on one stream, each on its own HIP stream so that their
    kernels overlap, or (one_graph) every shape's reconstruction in one HIP
    graph launch with one independent branch per plan (nlinv_reconstruct_multi,
    after each plan's gridding on the same stream).  groups: [(N, J, K, data)].
    Returns per-step ms."""
    runs = []
    for (n, j, k, data) in groups:
        B = len(data)
        plan = nl.Plan(n, j, k, U=U, batch=B, newton=M, cg=C)
        plan.set_graphs(graphs)
        traj = torch.from_numpy(np.stack([d[0] for d in data], axis=1)).cuda()
        y = torch.from_numpy(np.stack([d[1] for d in data], axis=1)).cuda()
        for t in range(U):
            plan.psf(traj[t, 0].contiguous(), t)
        st = torch.cuda.Stream() if concurrent else torch.cuda.current_stream()
        xs = [torch.empty(B, plan.X, dtype=torch.complex64, device="cuda") for _ in range(2)]
        z = torch.empty(B, j, n, n, dtype=torch.complex64, device="cuda")
        img = torch.empty(B, n, n, dtype=torch.float32, device="cuda")
        runs.append(dict(plan=plan, traj=traj, y=y, turn=data[0][2], st=st, xs=xs, z=z, img=img, B=B))
    torch.cuda.synchronize()

    def step(i):
        tns = []
        for r in runs:
            f = i % r["traj"].shape[0]
            tn = [int(r["turn"][f])] * r["B"]
            tns.append(tn)
            with torch.cuda.stream(r["st"]):
                r["plan"].grid(r["traj"][f], r["y"][f], turns=tn, z=r["z"])
                if not one_graph:
                    prev = None if i == 0 else r["xs"][(i - 1) & 1]
                    r["plan"].reconstruct(r["z"], tn, xprev=prev, xhat=r["xs"][i & 1], init=1 if i == 0 else 2,
                                          img=r["img"])
        if one_graph:
            nl.reconstruct_multi([r["plan"] for r in runs], [r["z"] for r in runs], tns,
                                 xprevs=[None if i == 0 else r["xs"][(i - 1) & 1] for r in runs],
                                 xhats=[r["xs"][i & 1] for r in runs], inits=[1 if i == 0 else 2] * len(runs),
                                 imgs=[r["img"] for r in runs])
        torch.cuda.synchronize()

    # graphs (the plans' own or the one-graph form) are captured per (turn,
    # buffer parity) argument set: frame 0 starts from the unit point, frames
    # 1 .. 2U see every set of the regularised frames, all before the clock
    if graphs or one_graph:
        warmup = max(warmup, 2 * U + 1)
    for i in range(warmup):
        step(i)
    per = []
    for i in range(warmup, warmup + steps):
        t0 = time.perf_counter()
        step(i)
        per.append((time.perf_counter() - t0) * 1e3)
    for r in runs:
        r["plan"].close()
    return per


def run_ragged_operator(torch, nl, batches=None, reps=30, warmup=5):
    """The CG operator of the three mixed shapes (one batched plan each, grids
    256, 320, 384; `batches` items each, default the mixed run's 5 / 6 / 5)
    applied with one ragged Toeplitz launch (nlinv_apply_normal_multi)
    against one nlinv_apply_normal per plan, all on one stream; ms per
    application of all three, host clock around synchronised GPU work."""
    import numpy as np
    from paper_1701_08361_amd import synth
    plans, xs, ps, turns = [], [], [], []
    shapes = [(n, j, k, b if batches is None else batches[i]) for i, (n, j, k, b) in enumerate(MIXED)]
    for i, (n, j, k, b) in enumerate(shapes):
        plan = nl.Plan(n, j, k, U=b, batch=b)
        for t in range(b):
            plan.psf(torch.from_numpy(synth.radial_trajectory(n, k, 2 * n, t, b)).cuda(), t)
        xs.append(torch.from_numpy(np.stack([synth.random_xhat(300 + 10 * i + t, plan.R, j, plan.Gc, 1.0, 0.3)
                                             for t in range(b)])).cuda())
        ps.append(torch.from_numpy(np.stack([synth.random_xhat(400 + 10 * i + t, plan.R, j, plan.Gc, 1.0, 0.3)
                                             for t in range(b)])).cuda())
        plans.append(plan)
        turns.append(list(range(b)))
    qs = [pl.empty(pl.B, pl.X) for pl in plans]

    def per_plan():
        for pl, t, x, p, q in zip(plans, turns, xs, ps, qs):
            pl.apply_normal(t, x, p, 0.1, q=q)

    def ragged():
        nl.apply_normal_multi(plans, turns, xs, [0.1] * len(plans), ps, qs)

    res = {}
    for name, fn in (("per_plan", per_plan), ("ragged", ragged), ("per_plan_again", per_plan),
                     ("ragged_again", ragged)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / reps * 1e3
    for pl in plans:
        pl.close()
    return {"batches": [b for (_, _, _, b) in shapes],
            "per_plan_ms": min(res["per_plan"], res["per_plan_again"]),
            "ragged_ms": min(res["ragged"], res["ragged_again"])}


def run_mixed_one_launch(torch, nl, groups, steps, warmup, graphs):
    """The same series in ONE batched plan on the largest shape's grid: every
    item of a smaller image side runs at gamma = G / (2 N) on that grid, its
    samples packed at the start of the plan's layout (nlinv_psf_samples) and
    its missing channels zero.  Returns per-step ms."""
    nmax = max(g[0] for g in groups)
    jmax = max(g[1] for g in groups)
    kmax = max(g[2] for g in groups)
    B = sum(len(g[3]) for g in groups)
    smax = kmax * 2 * nmax
    plan = nl.Plan(nmax, jmax, kmax, U=U * len(groups), batch=B, newton=M, cg=C)
    plan.set_graphs(graphs)
    F = min(len(g[3][0][2]) for g in groups)
    Y = torch.zeros(F, B, jmax, smax, dtype=torch.complex64, device="cuda")
    turn_of, i = [], 0
    for si, (n, j, k, data) in enumerate(groups):
        ns = k * 2 * n
        for t in range(U):
            tp = np.zeros((smax, 2), np.float32)
            tp[:ns] = data[0][0][t].reshape(ns, 2)
            plan.psf(torch.from_numpy(tp.reshape(kmax, 2 * nmax, 2)).cuda(), si * U + t, samples=ns)
        for d in data:
            Y[:, i, :j, :ns] = torch.from_numpy(d[1][:F]).cuda()
            turn_of.append((si, d[2]))
            i += 1
    traj = torch.zeros(B, kmax, 2 * nmax, 2, dtype=torch.float32, device="cuda")   # turns are cached: not read
    xs = [torch.empty(B, plan.X, dtype=torch.complex64, device="cuda") for _ in range(2)]
    z = torch.empty(B, jmax, plan.R, plan.R, dtype=torch.complex64, device="cuda")
    img = torch.empty(B, plan.R, plan.R, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def step(i):
        f = i % F
        tn = [si * U + int(tr[f]) for si, tr in turn_of]
        plan.grid(traj, Y[f], turns=tn, z=z)
        prev = None if i == 0 else xs[(i - 1) & 1]
        plan.reconstruct(z, tn, xprev=prev, xhat=xs[i & 1], init=1 if i == 0 else 2, img=img)
        torch.cuda.synchronize()

    if graphs:   # every (turn, buffer parity) argument set captured before the clock
        warmup = max(warmup, 2 * U + 1)
    for i in range(warmup):
        step(i)
    per = []
    for i in range(warmup, warmup + steps):
        t0 = time.perf_counter()
        step(i)
        per.append((time.perf_counter() - t0) * 1e3)
    plan.close()
    return per


def run_diff(torch, nl, data, steps, newton, cg):
    """Unrolled, checkpointed IRGNM of frame 0 (batch 1) with the loss
    ||image - phantom||^2 and its gradient with respect to the data, alpha_0
    and the Sobolev weight's a and l (at the plan's weight, a = 880, l = 16).
    Returns (forward ms, forward + backward ms) per step and the gradients."""
    from paper_1701_08361_amd import autograd as AG
    from paper_1701_08361_amd import unrolled as UR
    plan = nl.Plan(N, J, K, U=U, newton=newton, cg=cg)
    traj = torch.from_numpy(data[0][0][0:1]).cuda()
    y0 = torch.from_numpy(data[0][1][0:1]).cuda()
    target = torch.from_numpy(data[0][3]).cuda().float()
    plan.psf(traj[0], 0)
    fwd, tot, plain = [], [], []
    grads = {}
    for i in range(steps + 1):          # the plain solver on the same frame, same counts
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.reconstruct(plan.grid(traj, y0), [0])
        torch.cuda.synchronize()
        if i > 0:
            plain.append((time.perf_counter() - t0) * 1e3)
    for i in range(steps + 1):
        y = y0.clone().requires_grad_(True)
        a0 = torch.tensor(1.0, device="cuda", requires_grad=True)
        sa = torch.tensor(880.0, dtype=torch.float64, device="cuda", requires_grad=True)
        sl = torch.tensor(16.0, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = AG.Reweighted(plan, plan.G, plan.Gc, plan.R, J, sa, sl)
        x = UR.reconstruct(m, traj, y, N, newton=newton, cg_iters=cg, alpha0=a0, turns=[0])
        loss = ((UR.image(m, x, N)[0] - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if i > 0:                       # the first pass is a warm-up
            fwd.append((t1 - t0) * 1e3)
            tot.append((t2 - t0) * 1e3)
        grads = {"grad_norm_data": float(y.grad.abs().pow(2).sum().sqrt()), "grad_alpha0": float(a0.grad),
                 "grad_sobolev_a": float(sa.grad), "grad_sobolev_l": float(sl.grad)}
    plan.close()
    return fwd, tot, plain, grads


def run_autotune(torch, nl, data, frame_counts, graphs_allowed):
    """The autotuner's learning mode on the 160 px series for several series
    lengths: every setting (T frames per relaxed group = 1..8, A = 1, HIP
    graphs off / on, column-pass tiles of 8 or 4 columns) reconstructs the
    first `frames` frames, the database
    records each rate, and the worst and best settings are reported per
    length.  Rates include gridding and graph captures; plans and PSF kernels
    are built before the clock starts."""
    from paper_1701_08361_amd import autotune as AT
    traj_all = torch.from_numpy(data[0][0]).cuda()
    y_all = torch.from_numpy(data[0][1]).cuda()
    turns_all = [int(t) for t in data[0][2]]
    db = AT.TuningDB()
    rows = []
    for frames in frame_counts:
        frames = min(frames, traj_all.shape[0])
        p = dict(mode="single-slice", N=N, J=J, K=K, U=U, frames=frames, newton=M, cg=C)
        tuner = AT.Autotuner(db, learning=True, tiles=(8, 4), passes=(6, 4), splits=(0, 1))
        if not graphs_allowed:
            tuner.space = [c for c in tuner.space if not c["graphs"]]
        tuner.learn(p, lambda c: AT.run_series(nl, torch, traj_all[:frames], y_all[:frames],
                                               turns_all[:frames], c, M, C, U)[0])
        hits = db.lookup(p)
        (bc, bf), (wc, wf) = hits[0], hits[-1]
        rows.append({"frames": frames, "settings": len(hits),
                     "worst": dict(wc, fps=wf), "best": dict(bc, fps=bf),
                     "all": [[c["T"], c["graphs"], c["col_tile"], c["cg_passes"], c["fft_split"], round(f, 1)]
                             for c, f in hits]})
    return {"form": "learning mode over T = 1..8 frames per relaxed group (l = 5 strict frames first), A = 1, "
                    "HIP graphs off/on, column-pass tile schedule 8 or 4 columns per block, CG iteration of 6 or 4 "
                    "passes, Toeplitz-pass factorisation default or alternative; rate = frames / wall time of the "
                    "whole series (gridding + reconstruction); 'all' rows are [T, graphs, col_tile, cg_passes, "
                    "fft_split, fps]",
            "by_frames": rows}


def run_grid_choice(torch, nl, reps):
    """The grid-size lookup table of this GPU (G -> device time of one
    normal-operator application at batch 1, 10 channels, 15 spokes) over every
    grid side the library supports, and the grid it picks (gamma >= 1.4) for
    the image sides of Table oversampling_ratio."""
    from paper_1701_08361_amd import gridsize as GS
    grids = GS.supported_grids(nl)
    lut = GS.measure(nl, torch, grids, J=J, K=K, reps=reps)
    choice = {}
    for n in (128, 144, 160, 170, 256):
        try:
            g = GS.choose(n, lut)
            choice[str(n)] = {"G": g, "gamma": round(GS.gamma(n, g), 5)}
        except ValueError:
            choice[str(n)] = None
    # Table oversampling_ratio on this GPU where both grids are supported:
    # frames/s of the plain solve (7 x 20, each frame regularised to the
    # previous result) at the fixed gamma = 1.5 grid and at the chosen one
    from paper_1701_08361_amd import synth
    table = []
    for n in (128, 160, 170):
        g_fix = 3 * n
        row = {"N": n, "G_fixed": g_fix, "fps_fixed": None}
        if g_fix in grids:
            row["fps_fixed"] = round(_grid_fps(torch, nl, synth, n, g_fix), 1)
        g_opt = choice[str(n)]["G"] if choice[str(n)] else None
        row.update({"G_chosen": g_opt, "fps_chosen": round(_grid_fps(torch, nl, synth, n, g_opt), 1) if g_opt else None})
        if row["fps_fixed"] and row["fps_chosen"]:
            row["speedup"] = round(row["fps_chosen"] / row["fps_fixed"], 3)
        table.append(row)
    return {"us_per_normal_application": {str(g): round(t, 2) for g, t in lut.items()},
            "J": J, "K": K, "reps": reps, "choice_gamma_min_1_4": choice, "oversampling_table": table}


def _grid_fps(torch, nl, synth, n, G, frames=20):
    """Frames/s of the plain 7 x 20 solve of one synthetic 10-coil, 15-spoke
    frame on grid G, each frame regularised to the previous result."""
    s = synth.single_frame(seed=3, N=n, J=J, K=K)
    plan = nl.Plan(n, J, K, G=G, newton=M, cg=C)
    try:
        z = plan.grid(torch.from_numpy(s.traj).cuda(), torch.from_numpy(s.y).cuda(), turns=[0])
        xb = [plan.empty(1, plan.X) for _ in range(2)]
        img = torch.empty(1, plan.R, plan.R, dtype=torch.float32, device=plan.device)
        prev = None
        for f in range(frames + 3):
            if f == 3:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            plan.reconstruct(z, [0], xprev=prev, xhat=xb[f % 2], init=1 if prev is None else 2, img=img)
            prev = xb[f % 2]
        torch.cuda.synchronize()
        return frames / (time.perf_counter() - t0)
    finally:
        plan.close()


def run_pipeline(torch, raw, periods, period_ms, shared, graphs):
    """Slices of SLICES streamed through paper_1701_08361_amd.serve.Server at
    1000 / period_ms frames/s each: receive-channel samples in pinned host
    memory at arrival, then copy, compression, gridding, reconstruction and
    image copy-back.  shared: one copy and one solve stream for all slices
    (frames in arrival order); else per-slice streams.  Returns latencies (ms,
    image on the host - arrival) and wall ms."""
    from paper_1701_08361_amd import serve
    srv = serve.Server(budget_bytes=32 << 30, graphs=graphs, shared_streams=shared)
    names, host, trajs, turns = [], {}, {}, {}
    for (n, j, jp, k), (traj, y, turn) in zip(SLICES, raw):
        name = f"{n}px"
        tr = torch.from_numpy(traj).cuda()
        srv.admit(name, n, j, jp, k, U, tr[:U], torch.from_numpy(y[0]).cuda(), newton=M, cg=C)
        host[name] = torch.from_numpy(y).pin_memory()
        trajs[name], turns[name] = tr, turn
        names.append(name)
    F = min(len(turns[nm]) for nm in names)

    def period(i):
        evs = []
        for nm in names:
            f = i % F
            evs.append(srv.submit(nm, host[nm][f], trajs[nm][f], int(turns[nm][f]))[0])
        return evs

    for i in range(2 * U):                   # warm-up: graphs of every (turn, state buffer)
        period(i)
    srv.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    done = []
    for i in range(periods):
        arrival = i * period_ms
        now = (time.perf_counter() - t0) * 1e3
        if now < arrival:
            time.sleep((arrival - now) / 1e3)
        for ev in period(2 * U + i):
            done.append((ev, arrival))
    srv.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    lat = [start.elapsed_time(ev) - a for ev, a in done]
    for nm in names:
        srv.release(nm)
    return lat, wall


def pct(v, q):
    v = sorted(v)
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]


def roofline(kt_by_batch, head_batch):
    """Roofline object of the Toeplitz row pass (the dominant kernel).

    Per batch size B, from the HIP events carried in each launch's dispatch:
    algorithmic bytes of one launch = B J G R (8 + 8) + G^2 4 (the grid rows
    in and out at complex64 size, the PSF kernel rows once), divided by the
    average launch duration; frac = that rate / 8 TB/s.  The headline is the
    batch-`head_batch` launch; every batch size is listed on its own, never
    blended.  The grid is stored in float64, so the kernel moves
    `storage_factor` = 2 times the algorithmic bytes: `storage_gbs` is that
    rate."""
    by = {}
    for B, kt in sorted(kt_by_batch.items()):
        ms, n = kt.get("toeplitz_rows", (0.0, 0))
        if not n:
            continue
        t = ms / n / 1e3
        alg = kernel_bytes("toeplitz_rows", B, 1, 8)
        moved = kernel_bytes("toeplitz_rows", B, 1, 16)
        by[str(B)] = {"launches": n, "avg_launch_us": t * 1e6, "algorithmic_bytes": alg,
                      "achieved": alg / t / 1e9, "frac": alg / t / 1e9 / HBM_PEAK_GBS,
                      "storage_factor": moved / alg, "storage_gbs": moved / t / 1e9}
    head = by.get(str(head_batch))
    if head is None:
        return None
    meas = measured_traffic("toeplitz_rows")
    traffic = meas.get(head_batch) if meas else None
    return {"kernel": "toeplitz_rows", "batch": head_batch, "bound": "hbm", "achieved": head["achieved"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": head["frac"], "traffic": traffic,
            "algorithmic_bytes_per_launch": head["algorithmic_bytes"], "avg_launch_us": head["avg_launch_us"],
            "launches": head["launches"], "storage_factor": head["storage_factor"],
            "storage_gbs": head["storage_gbs"], "by_batch": by}


def copy_gbs(torch, mib=1024, reps=10):
    """Rate of a plain device-to-device copy of `mib` MiB (the runtime's copy
    kernel), bytes read plus bytes written per second: what the HBM delivers
    to a kernel that only streams, beside the published 8 TB/s.  1 GiB is four
    times the 256 MB Infinity Cache."""
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * n / t / 1e9


def cpu_baseline():
    """The FP64 oracle as it stands, on the host cores, on bounded samples:
      all threads : frame 0 of the 160 px series (exact gridding, PSF kernel,
                    7 x 20 IRGNM) -> `value` (frames/s);
      one thread  : the first Newton step (1 of 7, 20 CG) of the same frame,
                    scaled to frames/s by its share of the frame's operator
                    applications;
      64 px frame : the single 64 px, 8-coil, 13-spoke frame (7 x 10), in full,
                    all threads and one thread."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import nlinv_oracle as O
    from paper_1701_08361_amd import synth
    s = synth.real_time_series(seed=2, N=N, J=J, J_phys=J_PHYS, K=K, U=U, frames=1)
    g = O.Geometry.make(N, J)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    t0 = time.perf_counter()
    z = O.grid(s.y[0], s.traj[0], g.R)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    x = O.reconstruct(g, z, P, newton=M, cg_iters=C)
    dt = time.perf_counter() - t0
    assert np.isfinite(x).all()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.reconstruct(g, z, P, newton=1, cg_iters=C)
        dt1_step = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.grid(s.y[0], s.traj[0], g.R)
        O.psf_kernel(s.traj[0], g.R, g.G)
        dt1_prep = time.perf_counter() - t0
    dt1 = dt1_prep + M * dt1_step
    f1 = synth.single_frame(seed=1, N=64, J=8, K=13)
    g1 = O.Geometry.make(64, 8)

    def c1():
        t0 = time.perf_counter()
        z1 = O.grid(f1.y[0], f1.traj[0], g1.R)
        P1 = O.psf_kernel(f1.traj[0], g1.R, g1.G)
        O.reconstruct(g1, z1, P1, newton=7, cg_iters=10)
        return time.perf_counter() - t0
    c1_all = min(c1() for _ in range(3))
    with threadpool_limits(1):
        c1_one = min(c1() for _ in range(3))
    model = cpu_model()
    return {"value": 1.0 / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"1 frame (frame 0 of the 160px 10ch series: exact gridding, PSF kernel, 7x20 IRGNM) in "
                      f"{dt:.1f} s, {threads} BLAS threads on {os.cpu_count()} host CPUs ({model})",
            "one_core": {"value": 1.0 / dt1, "unit": "frames/s", "cores": 1,
                         "sample": f"gridding + PSF kernel ({dt1_prep:.1f} s) and Newton step 0 of 7 "
                                   f"(20 CG, {dt1_step:.1f} s) of frame 0, one thread; frame = prep + 7 steps"},
            "c1_64px": {"all_cores": {"value": 1.0 / c1_all, "unit": "frames/s", "cores": threads},
                        "one_core": {"value": 1.0 / c1_one, "unit": "frames/s", "cores": 1},
                        "sample": "the 64 px, 8-coil, 13-spoke frame (seed 1): exact gridding, PSF kernel, 7x10 "
                                  "IRGNM; best of 3"}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="timed frames of the plain series (the 100-frame series repeats; >= 1000 for p99)")
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed frames (with --graphs at least 2U, so that every (turn, buffer) graph is "
                         "captured before timing)")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--batched-plans", type=int, default=2,
                    help="the batched series as this many plans launched as one HIP graph (1: one plan)")
    ap.add_argument("--mode", choices=["both", "plain", "batched"], default="both")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graphs", action="store_true",
                    help="replay HIP graphs of the launch sequence (off by default: the autotuner measured "
                         "eager launches as fast or faster)")
    ap.add_argument("--kt-frames", type=int, default=3, help="frames with per-kernel event timing")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (reference kernel for HBM byte counters)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--relaxed-l", type=int, default=U, help="strict frames before relaxed coupling (l)")
    ap.add_argument("--relaxed-o", type=int, default=3, help="frames per relaxed group (o); 0 = skip")
    ap.add_argument("--source-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--serve-slices", type=int, default=4, help="slices streamed in the serving run (0 = skip)")
    ap.add_argument("--serve-periods", type=int, default=250, help="timed frame periods per slice")
    ap.add_argument("--hbm-batch", type=int, default=64,
                    help="batch of an extra run whose working set exceeds the 256 MB Infinity Cache (0 = skip)")
    ap.add_argument("--serve-fps", type=float, default=30.0, help="frames/s per slice")
    ap.add_argument("--diff-steps", type=int, default=2,
                    help="timed forward + backward passes of the unrolled 5 x 20 reconstruction (0 = skip)")
    ap.add_argument("--pipeline-periods", type=int, default=150,
                    help="timed periods of the streaming pipeline (4 slices, receive channels; 0 = skip)")
    ap.add_argument("--mixed-steps", type=int, default=10,
                    help="timed steps of the mixed-size run (3 shapes, 16 series; 0 = skip)")
    ap.add_argument("--autotune-frames", default="",
                    help="series lengths of an autotuning run (learning mode over all settings; '' = skip)")
    ap.add_argument("--col-tile", type=int, default=0, choices=[0, 4, 8],
                    help="columns per block of the CG column passes (0 = the library's choice)")
    ap.add_argument("--cg-passes-plain", type=int, default=4, choices=[0, 4, 6],
                    help="CG iteration form of the batch-1 plans (4: folded, measured faster at batch 1)")
    ap.add_argument("--cg-passes-serve", default="4,6",
                    help="CG iteration forms of the serving run's plain (batch 1) and batched policies")
    ap.add_argument("--cg-passes-relaxed", type=int, default=4, choices=[0, 4, 6],
                    help="CG iteration form of the relaxed-coupling plan (batch o, then one frame at a time)")
    ap.add_argument("--cg-passes-batched", type=int, default=6, choices=[0, 4, 6],
                    help="CG iteration form of the batched plans (6: fewer bytes, measured faster at batch 16)")
    ap.add_argument("--fft-split-plain", type=int, default=0, choices=[0, 1],
                    help="factorisation of the Toeplitz row pass in the batch-1 plans (0: the grid's default)")
    ap.add_argument("--fft-split-batched", type=int, default=0, choices=[0, 1],
                    help="factorisation of the Toeplitz row pass in the batched plans")
    ap.add_argument("--grid-lut-reps", type=int, default=0,
                    help="applications timed per grid side for the grid-size lookup table (0 = skip)")
    args = ap.parse_args()
    if args.batched_plans < 1 or args.batch % args.batched_plans:
        ap.error("--batched-plans must divide --batch")
    global COL_TILE
    COL_TILE = args.col_tile
    if args.source_hash:
        print(kernel_source_hash())
        return

    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (independent slices or series would shard "
                                   "one per GPU; no multi-GPU path is built)"}))
        sys.exit(2)

    frames_plain = max(U, min(100, args.warmup + args.steps + args.kt_frames))
    frames_batch = max(U, args.warmup + args.batch_steps + args.kt_frames)
    t_gen = time.perf_counter()
    plain_data = make_data([2], frames_plain, 1) if args.mode != "batched" else None
    batch_data = (make_data(list(range(2, 2 + args.batch)), frames_batch, args.workers)
                  if args.mode != "plain" else None)
    mixed_data = None
    if args.mixed_steps > 0 and args.mode == "both":
        frames_mixed = max(U, 2 * U + args.mixed_steps)
        seeds, jobs = 100, []
        for (n, j, k, ns) in MIXED:
            jobs.append([(seeds + q, frames_mixed, 1, n, j, k) for q in range(ns)])
            seeds += ns
        flat = [a for g in jobs for a in g]
        res = pool_map(_series, flat, args.workers)
        mixed_data, q = [], 0
        for (n, j, k, ns) in MIXED:
            mixed_data.append((n, j, k, res[q:q + ns]))
            q += ns
    raw_data = None
    if args.pipeline_periods > 0 and args.mode == "both":
        jobs = [(200 + q, 2 * U + 10, n, j, jp, k) for q, (n, j, jp, k) in enumerate(SLICES)]
        raw_data = pool_map(_raw_series, jobs, args.workers)
    t_gen = time.perf_counter() - t_gen

    cpu = None if args.no_cpu else cpu_baseline()

    import torch
    from paper_1701_08361_amd import nlinv as nl
    if not os.path.exists(nl.LIB_PATH):
        from paper_1701_08361_amd import build
        build.build(verbose=False)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nl.load()

    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    flags = 0
    KT_CLASSES = ["toeplitz_rows"]
    kt_by_batch = {}                     # batch -> {class: (ms, launches)}
    out = {"metric": "frames/sec + p99 frame latency, 160px 10ch NLINV, batched vs plain, 1 GPU",
           "unit": "frames/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "mixed", "data": "synthetic",
           "precision": {"storage": "c64 (data, gridded data, unknowns x_hat, coil images, channel products, "
                                    "PSF kernel f32)",
                         "operator_passes": "f64 arithmetic (registers, LDS) and f64 intermediates (coil rows, "
                                            "half-transformed grid)",
                         "cg_state": "f64 vectors (h, r, p, q), f64 dot products and scalars, f64 Newton update"}}
    img_strict = None
    if plain_data is not None:
        # frames 0 .. nwarm + steps - 1 of the strict series (run_mode's warm-up count)
        img_strict = torch.zeros((max(args.warmup, 2 * U) if args.graphs else args.warmup) + args.steps, N, N,
                                 dtype=torch.float32, device="cuda")
        per, total, kt = run_mode(torch, nl, plain_data, 1, args.steps, args.warmup, KT_CLASSES, args.kt_frames,
                                  args.graphs, img_store=img_strict, flags=flags, cg_passes=args.cg_passes_plain,
                                  fft_split=args.fft_split_plain)
        fps = args.steps / (total / 1e3)
        out.update({"value": fps, "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps,
                    "latency_ms": {"p50": pct(per, 50), "p99": pct(per, 99), "min": min(per)},
                    "effective_gbs": 1 * M * (C + 2) * compulsory_bytes_per_cg() / (total / args.steps / 1e3) / 1e9})
        kt_by_batch[1] = kt
    if plain_data is not None and args.relaxed_o > 0:
        l, o = args.relaxed_l, args.relaxed_o
        img_rel = torch.zeros_like(img_strict)
        nfr, total, per_g, n_end = run_relaxed(torch, nl, plain_data, args.steps, args.warmup, l, o,
                                               args.graphs, img_store=img_rel, cg_passes=args.cg_passes_relaxed)
        nmax = min(n_end, img_strict.shape[0])
        d = (img_rel[l + 1:nmax] - img_strict[l + 1:nmax]).flatten(1).norm(dim=1) / \
            img_strict[l + 1:nmax].flatten(1).norm(dim=1)
        d = d.cpu().tolist()
        out["relaxed"] = {"l": l, "o": o, "frames": nfr, "fps": nfr / (total / 1e3), "ms_per_frame": total / nfr,
                          "group_ms": {"p50": pct(per_g, 50), "p99": pct(per_g, 99), "min": min(per_g)},
                          "image_rel_diff_vs_strict": {"median": pct(d, 50), "max": max(d), "frames": len(d)}}
    if batch_data is not None:
        B = args.batch
        per, total, kt = run_mode(torch, nl, batch_data, B, args.batch_steps, args.warmup, KT_CLASSES,
                                  args.kt_frames, args.graphs, flags=flags, cg_passes=args.cg_passes_batched,
                                  fft_split=args.fft_split_batched)
        one_plan = {"fps": B * args.batch_steps / (total / 1e3), "ms_per_step": total / args.batch_steps,
                    "latency_ms": {"p50": pct(per, 50), "p99": pct(per, 99), "min": min(per)}}
        kt_by_batch[B] = kt
        P = args.batched_plans
        if P > 1:
            per, total = run_split(torch, nl, batch_data, B, P, args.batch_steps, args.warmup,
                                   cg_passes=args.cg_passes_batched, fft_split=args.fft_split_batched)
        out["batched"] = {"batch": B, "plans": P, "steps": args.batch_steps,
                          "fps": B * args.batch_steps / (total / 1e3),
                          "ms_per_step": total / args.batch_steps,
                          "latency_ms": {"p50": pct(per, 50), "p99": pct(per, 99), "min": min(per)},
                          "effective_gbs": B * M * (C + 2) * compulsory_bytes_per_cg() /
                                           (total / args.batch_steps / 1e3) / 1e9}
        if P > 1:
            out["batched"]["form"] = (f"{P} plans of {B // P} series, each step one HIP graph launch of all "
                                      "their reconstructions (nlinv_reconstruct_multi)")
            out["batched"]["one_plan"] = one_plan
        if plain_data is None:
            out.update({"value": out["batched"]["fps"], "steps": args.batch_steps, "warmup": args.warmup,
                        "ms_per_step": out["batched"]["ms_per_step"]})
    if batch_data is not None and args.hbm_batch > 0:
        # U2 of 64 items is 64 x 10 x 320 x 160 x 8 B = 262 MB (float32) / 524 MB (float64): the float64
        # launches' working set exceeds the 256 MB Infinity Cache, so their traffic reaches HBM
        hb = args.hbm_batch
        data_hb = [batch_data[i % len(batch_data)] for i in range(hb)]
        _, total_hb, kt = run_mode(torch, nl, data_hb, hb, 2, 0, KT_CLASSES, 1, args.graphs, flags=flags,
                                   cg_passes=args.cg_passes_batched, fft_split=args.fft_split_batched)
        kt_by_batch[hb] = kt
        out["hbm_check"] = {"batch": hb, "fps": hb * 2 / (total_hb / 1e3)}
    if batch_data is not None and args.serve_slices > 0:
        S = min(args.serve_slices, len(batch_data))
        forms = [int(v) for v in args.cg_passes_serve.split(",")]
        serving = {"slices": S, "fps_per_slice": args.serve_fps, "periods": args.serve_periods,
                   "cg_passes": {"plain": forms[0], "batched": forms[-1]}}
        for policy, cp in (("plain", forms[0]), ("batched", forms[-1])):
            lat, nfr, wall = run_serving(torch, nl, batch_data, S, args.serve_periods, 1e3 / args.serve_fps, policy,
                                         args.graphs, cg_passes=cp)
            serving[policy] = {"latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)},
                               "frames": nfr, "fps": nfr / (wall / 1e3)}
        out["serving"] = serving
    if plain_data is not None and args.diff_steps > 0:
        fwd, tot, plain, grads = run_diff(torch, nl, plain_data, args.diff_steps, 5, C)
        out["differentiation"] = {
            "form": "unrolled IRGNM in the Toeplitz form (gridded data, PSF convolution, hand-written backward), "
                    "5 Newton x 20 CG, checkpointed per Newton step, batch 1, 160 px 10 coils; "
                    "loss ||image - phantom||^2; gradients w.r.t. the data, alpha_0 and the Sobolev weight's "
                    "a and l (w = (1 + a|k|^2)^l at 880, 16); plain = gridding + the library's solver on the "
                    "same frame with the same counts",
            "forward_ms": pct(fwd, 50), "forward_backward_ms": pct(tot, 50), "plain_forward_ms": pct(plain, 50),
            "forward_over_plain": pct(fwd, 50) / pct(plain, 50), **grads}
    if raw_data is not None:
        pipe = {"slices": [{"N": n, "J": j, "J_phys": jp, "K": k} for (n, j, jp, k) in SLICES],
                "fps_per_slice": args.serve_fps, "periods": args.pipeline_periods,
                "steps": "pinned host samples -> copy -> channel compression -> gridding -> "
                         "reconstruction (7 x 20) -> image to host"}
        for name, shared in (("shared_streams", True), ("per_slice_streams", False)):
            lat, wall = run_pipeline(torch, raw_data, args.pipeline_periods, 1e3 / args.serve_fps, shared,
                                     args.graphs)
            pipe[name] = {"latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)},
                          "fps": len(lat) / (wall / 1e3)}
        out["serving_pipeline"] = pipe
    if plain_data is not None and args.autotune_frames:
        out["autotune"] = run_autotune(torch, nl, plain_data, [int(f) for f in args.autotune_frames.split(",")],
                                       args.graphs)
    if args.grid_lut_reps > 0:
        out["grid_choice"] = run_grid_choice(torch, nl, args.grid_lut_reps)
    if mixed_data is not None:
        nfr = sum(len(g[3]) for g in mixed_data)
        mixed = {"shapes": [{"N": n, "J": j, "K": k, "series": len(d)} for (n, j, k, d) in mixed_data],
                 "frames_per_step": nfr}
        for name, conc, one in (("one_stream", False, False), ("streams", True, False), ("one_graph", False, True)):
            per = run_mixed(torch, nl, mixed_data, args.mixed_steps, 2 * U, conc, args.graphs, one_graph=one)
            mixed[name] = {"fps": nfr / (sum(per) / len(per) / 1e3), "ms_per_step": {"p50": pct(per, 50),
                                                                                    "p99": pct(per, 99)}}
        mixed["one_graph"]["form"] = ("each shape's gridding, then every shape's reconstruction as one HIP graph "
                                      "launch with one branch per plan (nlinv_reconstruct_multi), all on one stream")
        per = run_mixed_one_launch(torch, nl, mixed_data, args.mixed_steps, 2 * U, args.graphs)
        mixed["one_launch"] = {"fps": nfr / (sum(per) / len(per) / 1e3),
                               "ms_per_step": {"p50": pct(per, 50), "p99": pct(per, 99)},
                               "form": "all series in one batched plan on the largest grid (smaller image "
                                       "sides at gamma = G / 2N, zero channels, packed samples)"}
        mixed["ragged_operator"] = {
            "form": "CG operator of the 3 mixed shapes (grids 256 / 320 / 384) on one stream: one "
                    "nlinv_apply_normal per plan, or nlinv_apply_normal_multi with one ragged persistent Toeplitz "
                    "launch (the tiles of every shape in one list, each shape on its own grid); ms per "
                    "application of all three",
            "runs": [run_ragged_operator(torch, nl), run_ragged_operator(torch, nl, batches=(1, 1, 1))]}
        out["mixed"] = mixed
    out["config"] = {"workload": "real-time series 160px (320 grid), 10 virtual coils, 15 spokes x 320, "
                                 "5 turns, 7 Newton x 20 CG, temporal regularisation",
                     "plain_batch": 1, "batched_batch": args.batch, "cg_passes_plain": args.cg_passes_plain,
                     "cg_passes_batched": args.cg_passes_batched, "cg_passes_relaxed": args.cg_passes_relaxed,
                     "fft_split_plain": args.fft_split_plain, "fft_split_batched": args.fft_split_batched,
                     "hip_graphs": args.graphs,
                     "data_gen_s": round(t_gen, 1)}
    if kt_by_batch:
        rl = roofline(kt_by_batch, args.batch if batch_data is not None else 1)
        if rl is not None:
            cg = copy_gbs(torch)
            rl["attainable"] = {"copy_gbs": cg, "storage_frac_of_copy": rl["storage_gbs"] / cg,
                                "form": "1 GiB device-to-device copy (read + written bytes per second)"}
        out["roofline"] = rl
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
