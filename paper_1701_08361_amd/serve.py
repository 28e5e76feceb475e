"""Streaming reconstruction of several slices (the real-time pipeline of
Sec. 3.1: data source -> preprocessing -> reconstruction -> postprocessing
-> sink), on one GPU.

Each admitted slice has its own plan (its shape), its own HIP streams (one
for host-to-device copies, one for the solve), its compression matrix, and
its previous-frame state kept on the device.  A frame arrives as
receive-channel samples in pinned host memory; submit() enqueues, without
blocking the host:

    copy stream:  raw samples -> device (pinned, asynchronous)
    solve stream: wait for the copy; channel compression; gridding;
                  reconstruction regularised to the slice's previous frame;
                  combined image -> pinned host buffer

so that the copy of a frame overlaps the solve of the previous one and the
slices' solves overlap each other.  Admission checks the device memory the
slice needs (plan workspace and buffers) against the server's budget.

Every step runs in the C-ABI library; this module only orders the calls and
owns the buffers.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

from . import nlinv


class BudgetError(RuntimeError):
    """Admitting the slice would exceed the server's device-memory budget."""


@dataclasses.dataclass
class _Slice:
    name: str
    plan: "nlinv.Plan"
    Jp: int
    cc: object
    copy_stream: object
    solve_stream: object
    yp: List[object]          # device raw samples, double buffered
    y: object
    z: object
    x: List[object]           # device state, ping-pong
    img_dev: object
    img_host: List[object]    # pinned host images, double buffered
    bytes: int
    frames: int = 0
    consumed: List[object] = dataclasses.field(default_factory=lambda: [None, None])


class Server:
    """Slices of different shapes reconstructed as their frames arrive."""

    def __init__(self, budget_bytes: int, graphs: bool = True, device: str = "cuda", shared_streams: bool = False):
        """shared_streams: every slice uses the same copy and solve streams, so
        frames are solved one at a time in arrival order (the plain,
        first-come-first-served pipeline); otherwise each slice has its own."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.used = 0
        self.graphs = graphs
        self.slices: Dict[str, _Slice] = {}
        self.shared = (torch.cuda.Stream(device=self.device), torch.cuda.Stream(device=self.device)) \
            if shared_streams else None

    # ------------------------------------------------------------------
    @staticmethod
    def slice_bytes(N: int, J: int, J_phys: int, K: int, U: int, newton: int, cg: int) -> int:
        """Device memory of one slice: plan workspace plus its buffers."""
        p = nlinv.make_params(N, J, K, U=U, newton=newton, cg=cg)
        sz = nlinv.sizes(p)
        S, X, R = sz["S"], sz["X"], sz["R"]
        bufs = 2 * J_phys * S * 8 + J * S * 8 + J * R * R * 8 + 2 * X * 8 + R * R * 4 + J * J_phys * 8
        return nlinv.workspace_size(p) + 256 + bufs

    def admit(self, name: str, N: int, J: int, J_phys: int, K: int, U: int, trajs, calib,
              newton: int = 7, cg: int = 20, cg_passes: int = 4):
        """Add a slice.  trajs: device [U][K][S_r][2] trajectories of its turns;
        calib: device [J_phys][S] calibration frame for the channel compression.
        cg_passes: CG iteration form of the slice's plan (one frame at a time:
        the four-pass form, measured faster at batch 1).
        Raises BudgetError (and allocates nothing) when the budget would be
        exceeded."""
        torch = self.torch
        if name in self.slices:
            raise ValueError(f"slice {name!r} already admitted")
        need = self.slice_bytes(N, J, J_phys, K, U, newton, cg)
        if self.used + need > self.budget:
            raise BudgetError(f"slice {name!r} needs {need} bytes, {self.budget - self.used} of the budget left")
        if self.shared is not None:
            copy_stream, solve_stream = self.shared
        else:
            copy_stream = torch.cuda.Stream(device=self.device)
            solve_stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(solve_stream):
            plan = nlinv.Plan(N, J, K, U=U, newton=newton, cg=cg, device=self.device, cg_passes=cg_passes)
            plan.set_graphs(self.graphs)
            for t in range(U):
                plan.psf(trajs[t].contiguous(), t)
            cc = plan.compression_matrix(calib.contiguous())
            S, X, R = plan.S, plan.X, plan.R
            dev = self.device
            yp = [torch.empty(1, J_phys, S, dtype=torch.complex64, device=dev) for _ in range(2)]
            y = torch.empty(1, J, S, dtype=torch.complex64, device=dev)
            z = torch.empty(1, J, R, R, dtype=torch.complex64, device=dev)
            x = [torch.empty(1, X, dtype=torch.complex64, device=dev) for _ in range(2)]
            img_dev = torch.empty(1, R, R, dtype=torch.float32, device=dev)
        img_host = [torch.empty(R, R, dtype=torch.float32, pin_memory=True) for _ in range(2)]
        solve_stream.synchronize()
        self.slices[name] = _Slice(name, plan, J_phys, cc, copy_stream, solve_stream, yp, y, z, x, img_dev,
                                   img_host, need)
        self.used += need
        return self.slices[name]

    def release(self, name: str):
        s = self.slices.pop(name)
        s.solve_stream.synchronize()
        s.plan.close()
        self.used -= s.bytes

    # ------------------------------------------------------------------
    def submit(self, name: str, yp_host, traj, turn: int):
        """Enqueue one frame of a slice: yp_host pinned [J_phys][S] receive
        samples, traj device [K][S_r][2] of turn `turn`.  Returns (event, image
        host tensor) — the image is valid once the event has completed."""
        torch = self.torch
        s = self.slices[name]
        k = s.frames
        buf = s.yp[k & 1]
        with torch.cuda.stream(s.copy_stream):
            if s.consumed[k & 1] is not None:       # frame k - 2 has left this buffer
                s.copy_stream.wait_event(s.consumed[k & 1])
            buf[0].copy_(yp_host, non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(s.copy_stream)
        with torch.cuda.stream(s.solve_stream):
            s.solve_stream.wait_event(copied)
            s.plan.compress(s.cc, buf, y=s.y)
            consumed = torch.cuda.Event()
            consumed.record(s.solve_stream)
            s.consumed[k & 1] = consumed
            s.plan.grid(traj[None], s.y, turns=[turn], z=s.z)
            prev = s.x[(k - 1) & 1] if k > 0 else None
            s.plan.reconstruct(s.z, [turn], xprev=prev, xhat=s.x[k & 1], init=1 if k == 0 else 2, img=s.img_dev)
            out = s.img_host[k & 1]
            out.copy_(s.img_dev[0], non_blocking=True)
            done = torch.cuda.Event(enable_timing=True)
            done.record(s.solve_stream)
        s.frames += 1
        return done, out

    def synchronize(self):
        for s in self.slices.values():
            s.copy_stream.synchronize()
            s.solve_stream.synchronize()
