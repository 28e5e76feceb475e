"""Seeded synthetic inputs for radial real-time NLINV.

This module is the only code shared by the FP64 oracle and the HIP path. It
produces *inputs* (trajectories and multi-channel k-space samples) and the
ground-truth objects they were synthesised from; it contains none of the
reconstruction arithmetic (no discrete Fourier operator, no gridding, no
point-spread function, no Sobolev weighting).

Acquisition (paper, Sec. 2.1 and Fig. "reorder"): U turns of K radial spokes;
spoke s of frame n lies at angle 2*pi*s/K + 2*pi*(n mod U)/(K*U), so that the
U turns together cover k-space uniformly.  Along a spoke there are S_r samples
with twofold readout oversampling, k_m = (m - S_r/2)/(2N) cycles/pixel, which
spans [-1/2, 1/2) when S_r = 2N.  Odd K only: with spokes over the full 2*pi,
an even K would place spoke s and s+K/2 on the same line.

Object: a continuous phantom made of filled ellipses (amplitudes add, as in
the classic head phantoms) multiplied by smooth coil sensitivities written as
finite 2D Fourier series with period L = 2R pixels.  The Fourier transform of
(ellipse x plane wave) is a shifted, phase-ramped jinc, so every k-space sample
is evaluated in closed form with the Bessel function J1.  No discretised image
model is used to make the data.

Channel compression (paper, Sec. 3.1, preprocessing stage): the physical
channels are compressed to J virtual channels with a PCA computed on the first
frame (the calibration phase) and applied to every frame.  This only prepares
the virtual-channel inputs of the reconstruction tests (numpy's SVD).  The
library's compression and the oracle's are checked against each other on the
receive channels returned with compress=False, never against this function.

Scaling and noise: each series is scaled by 100/||y_0|| (frame 0, all
channels), then complex Gaussian noise of standard deviation sigma
(sigma/sqrt(2) per real component) is added; samples are stored as complex64
and trajectories as float32.

Coordinates: image pixel (iy, ix) of an R x R image sits at (x, y) =
(ix - R/2, iy - R/2) pixels.  Trajectory arrays are [..., K, S_r, 2] with
[..., 0] = kx and [..., 1] = ky in cycles/pixel; the signal model is
y(k) = integral of u(r) exp(-i 2 pi k.r) dr.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
from scipy.special import j1 as _bessel_j1


# --------------------------------------------------------------------------
# acquisition
# --------------------------------------------------------------------------

def spoke_angles(K: int, turn: int, U: int) -> np.ndarray:
    """Angles of the K spokes of a frame acquired in turn `turn` (Fig. reorder:
    sigma = 2 pi / K between spokes, tau = 2 pi / (K U) between turns)."""
    s = np.arange(K, dtype=np.float64)
    return 2.0 * np.pi * s / K + 2.0 * np.pi * (turn % U) / (K * U)


def radial_trajectory(N: int, K: int, S_r: int, turn: int = 0, U: int = 1) -> np.ndarray:
    """float32 [K, S_r, 2] sample positions in cycles/pixel."""
    if K % 2 == 0:
        raise ValueError("odd spoke counts only (even K duplicates spokes over 2*pi)")
    theta = spoke_angles(K, turn, U)
    km = (np.arange(S_r, dtype=np.float64) - S_r / 2.0) / (2.0 * N)
    traj = np.empty((K, S_r, 2), dtype=np.float64)
    traj[:, :, 0] = np.cos(theta)[:, None] * km[None, :]
    traj[:, :, 1] = np.sin(theta)[:, None] * km[None, :]
    return traj.astype(np.float32)


# --------------------------------------------------------------------------
# phantom: filled ellipses
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Ellipse:
    cx: float     # centre, pixels
    cy: float
    a: float      # semi-axes, pixels
    b: float
    phi: float    # rotation, radians
    amp: float    # real amplitude


def ellipse_image(R: int, ells: List[Ellipse]) -> np.ndarray:
    """Pixel-centre samples of the phantom on the R x R grid (float64)."""
    c = np.arange(R, dtype=np.float64) - R / 2.0
    X, Y = np.meshgrid(c, c, indexing="xy")   # X[iy, ix] = x, Y[iy, ix] = y
    img = np.zeros((R, R), dtype=np.float64)
    for e in ells:
        dx, dy = X - e.cx, Y - e.cy
        u = (dx * np.cos(e.phi) + dy * np.sin(e.phi)) / e.a
        v = (-dx * np.sin(e.phi) + dy * np.cos(e.phi)) / e.b
        img += e.amp * ((u * u + v * v) <= 1.0)
    return img


def _ellipse_ft(kx: np.ndarray, ky: np.ndarray, e: Ellipse) -> np.ndarray:
    """Continuous Fourier transform of one filled ellipse at (kx, ky)."""
    u = e.a * (kx * np.cos(e.phi) + ky * np.sin(e.phi))
    v = e.b * (-kx * np.sin(e.phi) + ky * np.cos(e.phi))
    q = np.sqrt(u * u + v * v)
    safe = np.where(q > 1e-12, q, 1.0)
    jinc = np.where(q > 1e-12, _bessel_j1(2.0 * np.pi * safe) / safe, np.pi)
    return (e.amp * e.a * e.b) * jinc * np.exp(-2j * np.pi * (kx * e.cx + ky * e.cy))


# --------------------------------------------------------------------------
# coils: finite Fourier series with period L = 2R
# --------------------------------------------------------------------------

def _freq_grid(Q: int) -> np.ndarray:
    q = np.arange(-Q, Q + 1)
    qy, qx = np.meshgrid(q, q, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel()], axis=1).astype(np.float64)  # [(2Q+1)^2, 2]


def ring_gaussian_coeffs(J: int, R: int, Q: int = 4, width: float = 0.35,
                         radius: float = 0.45, phase: bool = True) -> np.ndarray:
    """Fourier coefficients [J, (2Q+1)^2] of smooth Gaussian-profile coils whose
    centres lie on a ring of radius `radius*R`; coil j carries the constant phase
    2 pi j / J.  Coefficients are those of a Gaussian of standard deviation
    `width*R`, truncated to |q|_inf <= Q (period L = 2R)."""
    L = 2.0 * R
    f = _freq_grid(Q) / L                                 # cycles/pixel
    s = width * R
    ang = 2.0 * np.pi * np.arange(J) / J
    centres = radius * R * np.stack([np.cos(ang), np.sin(ang)], axis=1)   # [J, 2]
    env = np.exp(-2.0 * np.pi ** 2 * s * s * np.sum(f * f, axis=1))      # [(2Q+1)^2]
    ph = np.exp(-2j * np.pi * (centres @ f.T))                             # [J, nq]
    coef = env[None, :] * ph
    if phase:
        coef = coef * np.exp(2j * np.pi * np.arange(J) / J)[:, None]
    # normalise so that each coil peaks near magnitude 1 inside the FOV
    coef /= np.sum(env)
    return coef


def random_smooth_coeffs(rng: np.random.Generator, J: int, Qr: int = 2) -> np.ndarray:
    """Random low-order Fourier series [J, (2Qr+1)^2]: CN(0,1) exp(-|q|^2/2)."""
    f = _freq_grid(Qr)
    w = np.exp(-0.5 * np.sum(f * f, axis=1))
    z = (rng.standard_normal((J, f.shape[0])) + 1j * rng.standard_normal((J, f.shape[0]))) / np.sqrt(2.0)
    return z * w[None, :]


def multiply_series(c1: np.ndarray, Q1: int, c2: np.ndarray, Q2: int):
    """Coefficients of the product of two Fourier series (2D convolution)."""
    n1, n2 = 2 * Q1 + 1, 2 * Q2 + 1
    Q = Q1 + Q2
    n = 2 * Q + 1
    J = c1.shape[0]
    a = c1.reshape(J, n1, n1)
    b = c2.reshape(J, n2, n2)
    out = np.zeros((J, n, n), dtype=np.complex128)
    for i in range(n2):
        for k in range(n2):
            out[:, i:i + n1, k:k + n1] += a * b[:, i:i + 1, k:k + 1]
    return out.reshape(J, n * n), Q


def coil_images(coef: np.ndarray, Q: int, R: int) -> np.ndarray:
    """Evaluate the coil Fourier series on the R x R pixel grid -> [J, R, R]."""
    L = 2.0 * R
    f = _freq_grid(Q) / L
    c = np.arange(R, dtype=np.float64) - R / 2.0
    ex = np.exp(2j * np.pi * np.outer(c, f[:, 0]))    # [R(x), nq]
    ey = np.exp(2j * np.pi * np.outer(c, f[:, 1]))    # [R(y), nq]
    # c_j(y, x) = sum_q coef[j,q] ey[y,q] ex[x,q]
    return np.einsum("jq,yq,xq->jyx", coef, ey, ex, optimize=True)


def kspace(traj: np.ndarray, ells: List[Ellipse], coef: np.ndarray, Q: int, R: int,
           static_cache: Optional[dict] = None, static_key=None,
           n_static: int = 0) -> np.ndarray:
    """Samples y[j, s] = FT[phantom * coil_j](k_s) for traj [K, S_r, 2] -> [J, K*S_r].

    The first `n_static` ellipses may be cached per `static_key` (e.g. the turn),
    because their transform depends only on the trajectory."""
    L = 2.0 * R
    f = _freq_grid(Q) / L
    k = traj.reshape(-1, 2).astype(np.float64)
    kx = k[None, :, 0] - f[:, 0:1]           # [nq, S]
    ky = k[None, :, 1] - f[:, 1:2]
    acc = None
    if static_cache is not None and static_key in static_cache:
        acc = static_cache[static_key].copy()
    else:
        acc = np.zeros(kx.shape, dtype=np.complex128)
        for e in ells[:n_static]:
            acc += _ellipse_ft(kx, ky, e)
        if static_cache is not None:
            static_cache[static_key] = acc.copy()
    for e in ells[n_static:]:
        acc += _ellipse_ft(kx, ky, e)
    return coef @ acc                         # [J, S]


def add_noise(rng: np.random.Generator, y: np.ndarray, sigma: float) -> np.ndarray:
    n = (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)) * (sigma / np.sqrt(2.0))
    return y + n


def pca_matrix(y0: np.ndarray, J: int) -> np.ndarray:
    """Compression matrix [J, J_phys]: conjugate-transposed top-J left singular
    vectors of the calibration frame y0 [J_phys, S]."""
    u, _, _ = np.linalg.svd(y0, full_matrices=False)
    return u[:, :J].conj().T


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Series:
    """A seeded frame series.  traj: float32 [F, K, S_r, 2]; y: complex64 [F, J, K*S_r];
    turn: int32 [F]; truth: float64 [F, R, R] phantom; coils: complex128 [J, R, R]
    (virtual-channel maps, before the data scaling)."""
    N: int
    K: int
    S_r: int
    U: int
    J: int
    traj: np.ndarray
    y: np.ndarray
    turn: np.ndarray
    truth: np.ndarray
    coils: np.ndarray
    scale: float


def _c1_ellipses(rng: np.random.Generator, R: int, n: int = 5) -> List[Ellipse]:
    out = []
    for _ in range(n):
        out.append(Ellipse(cx=rng.uniform(-0.3, 0.3) * R, cy=rng.uniform(-0.3, 0.3) * R,
                           a=rng.uniform(0.08, 0.3) * R, b=rng.uniform(0.08, 0.3) * R,
                           phi=rng.uniform(0.0, np.pi), amp=rng.uniform(0.2, 1.0)))
    return out


def single_frame(seed: int = 1, N: int = 64, J: int = 8, K: int = 13, S_r: Optional[int] = None,
                 sigma: float = 1e-3, n_ellipses: int = 5) -> Series:
    """Plain single frame: random ellipses, Gaussian-profile complex coils on a ring."""
    rng = np.random.default_rng(seed)
    S_r = 2 * N if S_r is None else S_r
    R = N
    ells = _c1_ellipses(rng, R, n_ellipses)
    Q = 4
    coef = ring_gaussian_coeffs(J, R, Q=Q)
    traj = radial_trajectory(N, K, S_r, 0, 1)
    y = kspace(traj, ells, coef, Q, R)
    scale = 100.0 / np.linalg.norm(y)
    y = add_noise(rng, y * scale, sigma)
    return Series(N=N, K=K, S_r=S_r, U=1, J=J, traj=traj[None], y=y[None].astype(np.complex64),
                  turn=np.zeros(1, np.int32), truth=ellipse_image(R, ells)[None],
                  coils=coil_images(coef, Q, R), scale=scale)


def _series_static(rng: np.random.Generator, R: int) -> List[Ellipse]:
    """Static part of the deforming phantom: a body ellipse with two features."""
    jit = lambda: rng.uniform(-0.02, 0.02) * R
    body = Ellipse(jit(), jit(), 0.42 * R, 0.36 * R, rng.uniform(-0.2, 0.2), 0.6)
    f1 = Ellipse(-0.2 * R + jit(), 0.15 * R + jit(), 0.06 * R, 0.09 * R, 0.3, -0.3)
    f2 = Ellipse(0.22 * R + jit(), 0.18 * R + jit(), 0.05 * R, 0.05 * R, 0.0, 0.4)
    return [body, f1, f2]


def _series_moving(R: int, n: int) -> Ellipse:
    """Inner ellipse of frame n; semi-axes vary as 1 +- 0.15 sin(2 pi n / 20)."""
    s = 0.15 * np.sin(2.0 * np.pi * n / 20.0)
    return Ellipse(0.1 * R, -0.05 * R, 0.14 * R * (1.0 + s), 0.11 * R * (1.0 - s), 0.5, 1.0)


def real_time_series(seed: int = 2, N: int = 160, J: int = 10, J_phys: int = 30, K: int = 15,
                     S_r: Optional[int] = None, U: int = 5, frames: int = 100,
                     sigma: float = 1e-3, compress: bool = True) -> Series:
    """Real-time series: deforming-ellipse phantom, J_phys random smooth coil maps
    (ring-Gaussian envelope x random low-order Fourier series) PCA-compressed to J
    virtual channels, K spokes per frame with U rotated turns.
    compress=False returns the J_phys receive channels instead (scaled by
    100 / ||frame 0||, noise added; J is ignored): the input of a pipeline that
    compresses the channels itself."""
    rng = np.random.default_rng(seed)
    S_r = 2 * N if S_r is None else S_r
    R = N
    Qe, Qr = 4, 2
    env = ring_gaussian_coeffs(J_phys, R, Q=Qe, phase=False)
    rnd = random_smooth_coeffs(rng, J_phys, Qr)
    coef, Q = multiply_series(env, Qe, rnd, Qr)
    base = _series_static(rng, R)
    cache: dict = {}
    y_all = np.empty((frames, J_phys, K * S_r), dtype=np.complex128)
    traj_all = np.empty((frames, K, S_r, 2), dtype=np.float32)
    truth = np.empty((frames, R, R), dtype=np.float64)
    turns = (np.arange(frames) % U).astype(np.int32)
    for n in range(frames):
        ells = base + [_series_moving(R, n)]
        traj = radial_trajectory(N, K, S_r, int(turns[n]), U)
        traj_all[n] = traj
        y_all[n] = kspace(traj, ells, coef, Q, R, static_cache=cache,
                          static_key=int(turns[n]), n_static=3)
        truth[n] = ellipse_image(R, ells)
    if compress:
        cc = pca_matrix(y_all[0], J)                   # calibration on frame 0
        yv = np.einsum("vp,fps->fvs", cc, y_all, optimize=True)
        coils = np.einsum("vp,pyx->vyx", cc, coil_images(coef, Q, R), optimize=True)
    else:
        J, yv, coils = J_phys, y_all, coil_images(coef, Q, R)
    scale = 100.0 / np.linalg.norm(yv[0])
    yv = add_noise(rng, yv * scale, sigma)
    return Series(N=N, K=K, S_r=S_r, U=U, J=J, traj=traj_all, y=yv.astype(np.complex64),
                  turn=turns, truth=truth, coils=coils, scale=scale)


def random_xhat(seed: int, R: int, J: int, Gc: int, scale_rho: float = 1.0,
                scale_c: float = 1.0) -> np.ndarray:
    """A seeded complex64 point of the unknown space [R*R + J*Gc*Gc] (image block
    followed by the coil-spectrum blocks) for operator tests."""
    rng = np.random.default_rng(seed)
    X = R * R + J * Gc * Gc
    v = (rng.standard_normal(X) + 1j * rng.standard_normal(X)) / np.sqrt(2.0)
    v[:R * R] *= scale_rho
    v[R * R:] *= scale_c
    return v.astype(np.complex64)


def random_samples(seed: int, J: int, S: int) -> np.ndarray:
    """Seeded complex64 radial-space vector [J, S]."""
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal((J, S)) + 1j * rng.standard_normal((J, S))) / np.sqrt(2.0)).astype(np.complex64)
