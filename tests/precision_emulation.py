"""CPU emulation of the rounding points of the GPU operator passes.

The GPU evaluates every operator application in passes with intermediates in
memory: the coil images c_j and the image rho are stored as complex64, the
coil-row buffer (the x-stage of W^-1 and W^-H) and the half-transformed grid
(the y-FFT of pad(u), the row-spectrum product, before the y-iFFT) as
complex128, the per-channel products conj(c_j) t_j as complex64.  This module
repeats the oracle's IRGNM (Sec. 2.2) with NumPy FFTs in FP64 and rounds the
values to complex64 at chosen points, so that the effect of a storage
precision on the reconstruction can be measured without a GPU.  It shares no
code with the HIP path; with no rounding point it reproduces the oracle.

Rounding points (names used in `rounding`):
  "co"    coil images c_j (once per Newton step)
  "x"     the unknowns x_hat (each Newton iterate)
  "pr"    the per-channel products conj(c_j) t_j
  "u1"    the x-stage of W^-1 (coil rows) and of W^-H
  "u2"    the half-transformed grid, before and after the row pass
`f32_steps` restricts "u1" / "u2" to the Newton steps m < f32_steps.

Run as a script to print the 160 px figures quoted in the design notes
(a few minutes per case; a comma-separated list of case numbers selects):
python tests/precision_emulation.py [0,1,...]
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import nlinv_oracle as O  # noqa: E402


def _r32(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def _dft(a, axis, inverse=False):
    """Unitary centred DFT along one axis (the oracle's convention)."""
    a = np.fft.ifftshift(a, axes=axis)
    a = (np.fft.ifft if inverse else np.fft.fft)(a, axis=axis, norm="ortho")
    return np.fft.fftshift(a, axes=axis)


def _pad(a, G, axis):
    n = a.shape[axis]
    o = G // 2 - n // 2
    shape = list(a.shape)
    shape[axis] = G
    out = np.zeros(shape, np.complex128)
    idx = [slice(None)] * a.ndim
    idx[axis] = slice(o, o + n)
    out[tuple(idx)] = a
    return out


def _crop(a, n, axis):
    G = a.shape[axis]
    o = G // 2 - n // 2
    idx = [slice(None)] * a.ndim
    idx[axis] = slice(o, o + n)
    return a[tuple(idx)]


class PassModel:
    """The operators of one Newton step, evaluated pass by pass."""

    def __init__(self, g: O.Geometry, P: np.ndarray, rounding: set):
        self.g, self.P, self.rnd = g, P, set(rounding)

    def _q(self, name, a):
        return _r32(a) if name in self.rnd else a

    def winv(self, chat):
        g = self.g
        a = _crop(_dft(_pad(chat / g.w, g.G, -1), -1, True), g.R, -1)      # x-stage (coil rows)
        a = self._q("u1", a)
        return _crop(_dft(_pad(a, g.G, -2), -2, True), g.R, -2)             # y-stage

    def winvh(self, v):
        g = self.g
        a = _crop(_dft(_pad(v, g.G, -2), -2), g.Gc, -2)
        a = self._q("u1", a)
        return _crop(_dft(_pad(a, g.G, -1), -1), g.Gc, -1) / g.w

    def toeplitz(self, u):
        g = self.g
        a = self._q("u2", _dft(_pad(u, g.G, -2), -2))                       # column pass
        a = _dft(_pad(a, g.G, -1), -1) * self.P[None]                        # row pass
        a = self._q("u2", _crop(_dft(a, -1, True), g.R, -1))
        return _crop(_dft(a, -2, True), g.R, -2)                             # column pass back

    def linearise(self, x):
        rho, chat = self.g.unpack(x)
        self.rho = self._q("x", rho)
        self.c = self._q("co", self.winv(self._q("x", chat)))

    def adjoint(self, t):
        top = self._q("pr", np.conj(self.c) * t).sum(0)
        return self.g.pack(top, self.winvh(np.conj(self.rho)[None] * t))

    def normal(self, p):
        drho, dchat = self.g.unpack(p)
        return self.adjoint(self.toeplitz(self.c * drho[None] + self.rho[None] * self.winv(dchat)))

    def rhs(self, x, xprev, z, alpha):
        return self.adjoint(z - self.toeplitz(self.rho[None] * self.c)) - alpha * (x - xprev)


def cg_replaced(apply_A, apply_exact, b, iters, every):
    """CG from h = 0 (the oracle's iteration) whose residual is recomputed as
    r = b - A_exact h after every `every` iterations, A_exact without the
    rounding points of the grid and the coil rows (residual replacement)."""
    h = np.zeros_like(b)
    r, p = b.copy(), b.copy()
    rr = O.rdot(r, r)
    for i in range(iters):
        q = apply_A(p)
        pq = O.rdot(p, q)
        a = rr / pq if pq != 0.0 else 0.0
        h = h + a * p
        r = r - a * q
        if (i + 1) % every == 0 and i + 1 < iters:
            r = b - apply_exact(h)
        rr_new = O.rdot(r, r)
        beta = rr_new / rr if rr != 0.0 else 0.0
        p = r + beta * p
        rr = rr_new
    return h


def reconstruct(g, z, P, rounding=(), f32_steps=None, x0=None, prevs=None, newton=7, cg_iters=20,
                replace_every=None):
    """IRGNM with the oracle's schedule; prevs[m] is the regularisation target
    of Newton step m (default: the start for every step).  replace_every: CG
    with residual replacement (cg_replaced) every that many iterations."""
    x = g.initial() if x0 is None else np.asarray(x0, np.complex128).copy()
    prevs = prevs or [x.copy()] * newton
    for m, alpha in enumerate(O.alpha_schedule(newton)):
        rnd = set(rounding)
        if f32_steps is not None and m >= f32_steps:
            rnd -= {"u1", "u2"}
        model = PassModel(g, P, rnd)
        model.linearise(x)
        b = model.rhs(x, prevs[m], z, alpha)
        A = lambda p: model.normal(p) + alpha * p  # noqa: E731
        if replace_every:
            exact = PassModel(g, P, rnd - {"u1", "u2"})
            exact.rho, exact.c = model.rho, model.c
            x = x + cg_replaced(A, lambda p: exact.normal(p) + alpha * p, b, cg_iters, replace_every)
        else:
            x = x + O.cg(A, b, cg_iters)
        if "x" in rnd:
            x = _r32(x)
    return x


def errors(g, x, ref):
    """Relative L2 of the combined image and of rho c_j against a reference."""
    e_img = np.linalg.norm(O.image(g, x) - O.image(g, ref)) / np.linalg.norm(O.image(g, ref))
    e_rc = np.linalg.norm(O.coil_images(g, x) - O.coil_images(g, ref)) / np.linalg.norm(O.coil_images(g, ref))
    return float(e_img), float(e_rc)


def main():
    from paper_1701_08361_amd import synth
    ser = synth.real_time_series(seed=2, frames=3)
    g = O.Geometry.make(160, 10)
    zs = [O.grid(ser.y[f], ser.traj[f], g.R) for f in range(3)]
    Ps = [O.psf_kernel(ser.traj[f], g.R, g.G) for f in range(3)]
    r0 = O.reconstruct(g, zs[0], Ps[0], newton=7, cg_iters=20)
    r1 = O.reconstruct(g, zs[1], Ps[1], xprev=r0, x0=r0, newton=7, cg_iters=20)
    x6 = O.reconstruct(g, zs[2], Ps[2], xprev=r0, x0=r0, newton=6, cg_iters=20)
    r2 = x6 + O.newton_step(g, x6, r1, zs[2], Ps[2], O.alpha_schedule(7)[6], 20)
    base = {"co", "x", "pr"}
    cases = [("complex64 coil images, unknowns, channel products (the library)", base, None, None),
             ("+ complex64 half-transformed grid in every step", base | {"u2"}, None, None),
             ("+ complex64 half-transformed grid in steps 0..5", base | {"u2"}, 6, None),
             ("+ complex64 coil rows in every step", base | {"u1"}, None, None),
             ("+ complex64 half-transformed grid, FP64 residual replacement every 5 CG iterations",
              base | {"u2"}, None, 5)]
    if len(sys.argv) > 1:
        cases = [cases[int(i)] for i in sys.argv[1].split(",")]
    for name, rnd, fs, rep in cases:
        e0 = reconstruct(g, zs[0], Ps[0], rnd, fs, replace_every=rep)
        e1 = reconstruct(g, zs[1], Ps[1], rnd, fs, x0=e0, prevs=[e0] * 7, replace_every=rep)
        e2 = reconstruct(g, zs[2], Ps[2], rnd, fs, x0=e0, prevs=[e0] * 6 + [e1], replace_every=rep)
        out = [errors(g, a, b) for a, b in ((e0, r0), (e1, r1), (e2, r2))]
        labels = ("frame 0", "frame 1 (from frame 0)", "relaxed frame 2 (steps 0..5 from frame 0)")
        print(f"{name}: " + "; ".join(f"{lab} image {a:.1e} rho.c {b:.1e}" for lab, (a, b) in zip(labels, out)),
              flush=True)


if __name__ == "__main__":
    main()
