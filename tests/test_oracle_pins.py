"""Pins of the FP64 oracle against things other than itself: closed forms,
textbook library routines, brute force on tiny inputs, exact algebraic
identities of the method and numbers printed in the paper.

Each test names the passage it follows.  Sizes are tiny so the whole file
runs in seconds on the CPU.
"""
import os

import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def tiny_geometry(N=8, J=2, K=5, seed=0):
    g = O.Geometry.make(N, J)
    traj = synth.radial_trajectory(N, K, 2 * N, 0, 1).astype(np.float64)
    rng = np.random.default_rng(seed)
    x = crand(rng, g.X)
    return g, traj, rng, x


# --------------------------------------------------------------------------
# uniform DFT: textbook special case, Parseval, inverse
# --------------------------------------------------------------------------

@pytest.mark.parametrize("G", [8, 16, 20, 24])
def test_dense_dft_matches_numpy_fft(G):
    """F_u (unitary, centred) equals numpy's FFT with centring shifts."""
    rng = np.random.default_rng(1)
    a = crand(rng, G, G)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(a), norm="ortho"))
    assert rel(O.fft2u(a), ref) < 1e-13
    refi = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(a), norm="ortho"))
    assert rel(O.ifft2u(a), refi) < 1e-13


def test_parseval_and_inverse():
    rng = np.random.default_rng(2)
    a = crand(rng, 3, 16, 16)
    A = O.fft2u(a)
    assert abs(np.linalg.norm(A) - np.linalg.norm(a)) / np.linalg.norm(a) < 1e-13
    assert rel(O.ifft2u(A), a) < 1e-13


def test_pad_crop_adjoint():
    rng = np.random.default_rng(3)
    a, b = crand(rng, 6, 6), crand(rng, 16, 16)
    assert abs(np.vdot(O.pad(a, 16), b) - np.vdot(a, O.crop(b, 6))) < 1e-12
    assert rel(O.crop(O.pad(a, 16), 6), a) == 0.0


# --------------------------------------------------------------------------
# non-uniform DFT: brute force and the Cartesian special case
# --------------------------------------------------------------------------

def test_nudft_matches_dense_matrix():
    """Separable evaluation == dense S x R^2 matrix (brute force, R = 8)."""
    g, traj, rng, _ = tiny_geometry()
    u = crand(rng, g.R, g.R)
    E = O.nudft_matrix(traj, g.R)
    assert rel(O.nudft(u, traj), E @ u.ravel()) < 1e-12
    v = crand(rng, E.shape[0])
    assert rel(O.nudft_adjoint(v, traj, g.R), (E.conj().T @ v).reshape(g.R, g.R)) < 1e-12


def test_nudft_on_cartesian_grid_is_the_fft():
    """With samples on the Cartesian grid k = m/R the NUDFT is numpy's unitary
    ("ortho"), centred 2D FFT: pins the sign (exp(-i 2 pi k.r)), the x/y order,
    the centring and the 1/R scale."""
    R = 8
    m = O.centred(R) / R
    KY, KX = np.meshgrid(m, m, indexing="ij")
    traj = np.stack([KX.ravel(), KY.ravel()], axis=1)
    rng = np.random.default_rng(4)
    u = crand(rng, R, R)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u), norm="ortho"))
    assert rel(O.nudft(u, traj).reshape(R, R), ref) < 1e-12
    # unitary: the adjoint inverts it
    assert rel(O.nudft_adjoint(O.nudft(u, traj), traj, R), u) < 1e-12


# --------------------------------------------------------------------------
# PSF convolution == F^H F (Sec. 2.2 and its footnote; Fig. flow)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("K", [5, 7])
def test_toeplitz_equals_EhE_bruteforce(K):
    N = 8
    g = O.Geometry.make(N, 1)
    traj = synth.radial_trajectory(N, K, 2 * N, 1, 3).astype(np.float64)
    P = O.psf_kernel(traj, g.R, g.G)
    E = O.nudft_matrix(traj, g.R)
    rng = np.random.default_rng(5)
    u = crand(rng, g.R, g.R)
    ref = (E.conj().T @ (E @ u.ravel())).reshape(g.R, g.R)
    assert rel(O.toeplitz(u, P), ref) < 1e-12


def test_psf_kernel_is_real_and_lag_R_matters():
    N = 8
    g = O.Geometry.make(N, 1)
    traj = synth.radial_trajectory(N, 5, 2 * N, 0, 1).astype(np.float64)
    P = O.psf_kernel(traj, g.R, g.G, keep_imag=True)
    assert np.max(np.abs(P.imag)) < 1e-11 * np.max(np.abs(P.real))
    # keeping the lag -R row/column (never used by FOV differences) breaks realness
    k = traj.reshape(-1, 2)
    d = np.arange(-g.R, g.R).astype(np.float64)
    full = np.exp(2j * np.pi * np.outer(k[:, 1], d)).T @ np.exp(2j * np.pi * np.outer(k[:, 0], d))
    Pf = g.G * O.fft2u(full)
    assert np.max(np.abs(Pf.imag)) > 1e-3 * np.max(np.abs(Pf.real))
    # and P is indefinite: there is no sqrt(P) factorisation of F^H F
    assert P.real.min() < 0 < P.real.max()


def test_cartesian_full_coverage_gives_scaled_identity():
    """All R^2 FOV frequencies sampled once -> psf = delta -> T = I."""
    R = 8
    m = O.centred(R) / R
    KY, KX = np.meshgrid(m, m, indexing="ij")
    traj = np.stack([KX.ravel(), KY.ravel()], axis=1)
    lag = O.psf_lags(traj, R)
    expect = np.zeros_like(lag)
    expect[R - 1, R - 1] = 1.0
    assert np.max(np.abs(lag - expect)) < 1e-10
    P = O.psf_kernel(traj, R, 2 * R)
    rng = np.random.default_rng(6)
    u = crand(rng, R, R)
    assert rel(O.toeplitz(u, P), u) < 1e-12


def test_wider_field_of_view_keeps_pixel_positions():
    """gamma > 1 (Sec. 3.2): G = 2 gamma N widens the reconstructed field of
    view to R' = G/2 > N around the same pixels.  The image padded into the
    wider FOV gives the same samples, up to the unitary scale 1/R; gridding
    onto the wider FOV holds the narrow one in its centre; the PSF of the
    narrow FOV is the centre of the wide one (all up to that scale)."""
    N, Rw, K = 8, 12, 5
    traj = synth.radial_trajectory(N, K, 2 * N, 0, 1).astype(np.float64)
    rng = np.random.default_rng(7)
    u = crand(rng, N, N)
    assert rel(Rw * O.nudft(O.pad(u, Rw), traj), N * O.nudft(u, traj)) < 1e-12
    y = crand(rng, 2, traj.size // 2)
    assert rel(Rw * O.crop(O.grid(y, traj, Rw), N), N * O.grid(y, traj, N)) < 1e-12
    o = Rw - N
    wide = O.psf_lags(traj, Rw)[o:o + 2 * N - 1, o:o + 2 * N - 1]
    assert rel(Rw ** 2 * wide, N ** 2 * O.psf_lags(traj, N)) < 1e-12


def test_gridding_is_adjoint_nudft():
    g, traj, rng, _ = tiny_geometry()
    y = crand(rng, 2, traj.size // 2)
    E = O.nudft_matrix(traj, g.R)
    z = O.grid(y, traj, g.R)
    for j in range(2):
        assert rel(z[j].ravel(), E.conj().T @ y[j]) < 1e-12


# --------------------------------------------------------------------------
# Sobolev weighting (Sec. 3.2, Fig. weight_func) and size arithmetic
# --------------------------------------------------------------------------

def test_sobolev_weight_printed_values():
    """w(k) = (1 + 880|k|^2)^16 on k in (-1/2, 1/2): w(0) = 1, w(1/2 on an axis) = 221^16."""
    G = 512
    w_full = O.sobolev_weight(G, G)                  # uncropped, Fig. weight_func grid
    c = G // 2
    assert w_full[c, c] == 1.0
    assert w_full[c, 0] == pytest.approx(221.0 ** 16, rel=1e-12)   # k_x = -1/2
    assert 221.0 ** 16 == pytest.approx(3.24e37, rel=1e-2)
    # cropped to G/4 (25 %): edge k = 1/8 -> 14.75^16, corner -> 28.5^16
    w = O.sobolev_weight(G, G // 4)
    assert w[0, G // 8] == pytest.approx(14.75 ** 16, rel=1e-12)
    assert w[0, 0] == pytest.approx(28.5 ** 16, rel=1e-12)
    assert 1.0 / w[0, 0] == pytest.approx(5.3e-24, rel=2e-2)


def _printed_grid_sizes():
    path = os.path.join(os.path.dirname(__file__), "golden", "grid_sizes.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            n, gf, gam, g, gcf, gc = line.split()
            rows.append((int(n), int(gf), float(gam), int(g), int(gcf), int(gc)))
    return rows


def test_printed_grid_sizes_fixture_is_complete():
    assert [r[0] for r in _printed_grid_sizes()] == [128, 144, 160, 170, 256]


@pytest.mark.parametrize("N,G_fixed,gamma,G,Gc_full,Gc", _printed_grid_sizes())
def test_grid_sizes_from_tables(N, G_fixed, gamma, G, Gc_full, Gc):
    """Tables oversampling_ratio and tiny: G = 2 gamma N (rounded; gamma = 1.5
    for the fixed column), the uncropped coil grid is G, and the oracle's
    cropped coil grid is G_c = floor(G / 4)."""
    assert round(2 * 1.5 * N) == G_fixed
    assert round(2 * gamma * N) == G
    assert Gc_full == G
    R, G2, Gc2 = O.sizes(N, G)
    assert (G2, Gc2) == (G, Gc) and R == G // 2 and R >= N


def test_winv_adjoint_pair():
    g, _, rng, _ = tiny_geometry(N=8)
    a = crand(rng, g.J, g.Gc, g.Gc)
    b = crand(rng, g.J, g.R, g.R)
    lhs = np.vdot(O.winv(a, g.G, g.R, g.w), b)
    rhs = np.vdot(a, O.winvh(b, g.G, g.Gc, g.w))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _weight_closed_form(ky, kx, G):
    """w(k) = (1 + 880 |k|^2)^16 at k = kappa / G (Fig. weight_func), written out
    here rather than taken from the oracle."""
    return (1.0 + 880.0 * (ky * ky + kx * kx) / float(G * G)) ** 16


@pytest.mark.parametrize("N,G", [(8, 16), (12, 24), (8, 20)])
def test_winv_of_a_spectral_spike_is_a_weighted_plane_wave(N, G):
    """Closed form of the coil synthesis W^-1 (Sec. 2.2, change of variables
    x_hat = W x; Fig. weight_func): a single coil coefficient c_hat = delta at
    the centred frequency kappa gives, on the field of view,
        c(r) = exp(+i 2 pi kappa . r / G) / (G w(kappa)),
    because F_u^-1 carries 1/G per 2D transform and W divides by w, not w^2 or
    sqrt(w).  Every frequency of the G_c x G_c block is checked, on an odd G_c
    (G = 20) as well."""
    R, G, Gc = O.sizes(N, G)
    w = O.sobolev_weight(G, Gc)
    cs = O.centred(R).astype(np.float64)
    Y, X = np.meshgrid(cs, cs, indexing="ij")
    worst = 0.0
    for iy, ky in enumerate(O.centred(Gc)):
        for ix, kx in enumerate(O.centred(Gc)):
            chat = np.zeros((1, Gc, Gc), complex)
            chat[0, iy, ix] = 1.0
            got = O.winv(chat, G, R, w)[0]
            ref = np.exp(2j * np.pi * (kx * X + ky * Y) / G) / (G * _weight_closed_form(ky, kx, G))
            worst = max(worst, rel(got, ref))
    assert worst < 1e-12


def _dirichlet(d, R, G):
    """sum over x = -floor(R/2) .. R - 1 - floor(R/2) of exp(-i 2 pi d x / G), by the geometric series."""
    a = -(R // 2)
    if d % G == 0:
        return complex(R)
    q = np.exp(-2j * np.pi * d / G)
    return q ** a * (1.0 - q ** R) / (1.0 - q)


@pytest.mark.parametrize("N,G", [(8, 16), (12, 24), (8, 20)])
def test_winvh_of_a_plane_wave_closed_form(N, G):
    """Closed form of W^-H (the adjoint coil synthesis of the normal-operator
    equation, Sec. 2.2): for the plane wave v(r) = exp(+i 2 pi kappa0 . r / G) on
    the field of view,
        (W^-H v)(kappa) = D(kappa_y - kappa0_y) D(kappa_x - kappa0_x) / (G w(kappa))
    with D the geometric sum over the R field-of-view coordinates; at kappa =
    kappa0 this is R^2 / (G w(kappa0))."""
    R, G, Gc = O.sizes(N, G)
    w = O.sobolev_weight(G, Gc)
    cs = O.centred(R).astype(np.float64)
    Y, X = np.meshgrid(cs, cs, indexing="ij")
    kc = O.centred(Gc)
    wc = np.array([[_weight_closed_form(ky, kx, G) for kx in kc] for ky in kc])
    worst = 0.0
    for k0y in (kc[0], 0, kc[-1]):
        for k0x in (kc[0], 1, kc[-1]):
            v = np.exp(2j * np.pi * (k0x * X + k0y * Y) / G)
            got = O.winvh(v[None], G, Gc, w)[0]
            # undo the closed-form 1 / (G w) and compare with the geometric sums; the
            # weights span 20 orders of magnitude, so the comparison is made on the
            # unweighted values, whose rounding is relative to their peak R^2
            dd = np.array([[_dirichlet(ky - k0y, R, G) * _dirichlet(kx - k0x, R, G) for kx in kc] for ky in kc])
            worst = max(worst, np.abs(got * G * wc - dd).max() / (R * R))
            iy, ix = list(kc).index(k0y), list(kc).index(k0x)
            assert abs(got[iy, ix] - R * R / (G * wc[iy, ix])) < 1e-12 * abs(got[iy, ix])
    assert worst < 1e-12


# --------------------------------------------------------------------------
# operator identities (Sec. 2.2: F = script-F o C, derivative and adjoint)
# --------------------------------------------------------------------------

def scaled_point(g, rng):
    """A point whose coil block is O(1) after W^-1 (spectra scaled by the weight)."""
    rho = crand(rng, g.R, g.R)
    chat = crand(rng, g.J, g.Gc, g.Gc) * g.w[None]
    return g.pack(rho, chat)


def test_DF_DFH_adjoint():
    g, traj, rng, _ = tiny_geometry(N=8, J=3, K=7)
    x, u = scaled_point(g, rng), scaled_point(g, rng)
    v = crand(rng, g.J, traj.size // 2)
    lhs = np.vdot(O.DF_hat(g, x, u, traj), v)
    rhs = np.vdot(u, O.DFH_hat(g, x, v, traj))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_F_is_bilinear_so_DF_is_exact():
    """F_hat(x + u) - F_hat(x) - DF_x u = F_hat(u) and the central difference equals DF_x u."""
    g, traj, rng, _ = tiny_geometry(N=8, J=2, K=5)
    x, u = scaled_point(g, rng), scaled_point(g, rng)
    Fx, Fu, Fxu = (O.F_hat(g, v, traj) for v in (x, u, x + u))
    DFu = O.DF_hat(g, x, u, traj)
    assert rel(Fxu - Fx - DFu, Fu) < 1e-12
    eps = 0.37
    cd = (O.F_hat(g, x + eps * u, traj) - O.F_hat(g, x - eps * u, traj)) / (2 * eps)
    assert rel(cd, DFu) < 1e-12
    # F_hat(x) = DF_x(x) / 2 (homogeneous of degree two)
    assert rel(O.DF_hat(g, x, x, traj) / 2, Fx) < 1e-12


def test_normal_operator_toeplitz_vs_explicit_and_hermitian_psd():
    g, traj, rng, _ = tiny_geometry(N=8, J=2, K=7)
    P = O.psf_kernel(traj, g.R, g.G)
    x, p, q = scaled_point(g, rng), crand(rng, g.X), crand(rng, g.X)
    Ap = O.normal(g, x, p, P)
    assert rel(Ap, O.normal_explicit(g, x, p, traj)) < 1e-11
    Aq = O.normal(g, x, q, P)
    assert abs(np.vdot(Ap, q) - np.vdot(p, Aq)) < 1e-11 * abs(np.vdot(Ap, q))
    assert np.real(np.vdot(p, Ap)) > 0


# --------------------------------------------------------------------------
# CG and the Newton step against dense linear algebra
# --------------------------------------------------------------------------

def dense_op(apply, n):
    cols = [apply(np.eye(n, dtype=np.complex128)[:, i]) for i in range(n)]
    return np.stack(cols, axis=1)


def test_cg_solves_the_newton_system():
    g, traj, rng, _ = tiny_geometry(N=8, J=2, K=5)
    P = O.psf_kernel(traj, g.R, g.G)
    x = scaled_point(g, rng) * 0.05
    alpha = 0.5
    A = dense_op(lambda p: O.normal(g, x, p, P), g.X) + alpha * np.eye(g.X)
    b = crand(rng, g.X)
    ref = np.linalg.solve(A, b)
    h = O.cg(lambda p: O.normal(g, x, p, P) + alpha * p, b, 300)
    assert rel(h, ref) < 1e-9


def test_newton_step_is_regularised_least_squares():
    """h minimises ||DF h - (y - F_hat x)||^2 + alpha ||h + x - x_prev||^2 (IRGNM update)."""
    g, traj, rng, _ = tiny_geometry(N=8, J=2, K=5)
    P = O.psf_kernel(traj, g.R, g.G)
    x = scaled_point(g, rng) * 0.05
    xprev = scaled_point(g, rng) * 0.05
    y = crand(rng, g.J, traj.size // 2)
    alpha = 0.25
    Jac = dense_op(lambda d: O.DF_hat(g, x, d, traj).ravel(), g.X)
    lhs = np.concatenate([Jac, np.sqrt(alpha) * np.eye(g.X)])
    rhs = np.concatenate([(y - O.F_hat(g, x, traj)).ravel(), -np.sqrt(alpha) * (x - xprev)])
    ref = np.linalg.lstsq(lhs, rhs, rcond=None)[0]
    z = O.grid(y, traj, g.R)
    h = O.newton_step(g, x, xprev, z, P, alpha, 300)
    assert rel(h, ref) < 1e-8


def test_first_newton_step_leaves_rho_unchanged():
    """From x_0 = (rho = 1, c = 0) the image block of A and of the right-hand side
    vanish (c = 0), so h_rho = 0 exactly in step 0."""
    s = synth.single_frame(seed=3, N=16, J=3, K=5)
    g = O.Geometry.make(16, 3)
    traj = s.traj[0]
    P = O.psf_kernel(traj, g.R, g.G)
    z = O.grid(s.y[0], traj, g.R)
    x0 = g.initial()
    h = O.newton_step(g, x0, x0, z, P, 1.0, 6)
    assert np.all(h[:g.R * g.R] == 0)
    assert np.linalg.norm(h[g.R * g.R:]) > 0


def test_zero_data_is_a_fixed_point():
    g = O.Geometry.make(8, 2)
    traj = synth.radial_trajectory(8, 5, 16, 0, 1)
    P = O.psf_kernel(traj, g.R, g.G)
    z = np.zeros((2, g.R, g.R), np.complex128)
    x = O.reconstruct(g, z, P, newton=3, cg_iters=4)
    assert np.array_equal(x, g.initial())


def test_alpha_schedule():
    assert O.alpha_schedule(4) == [1.0, 0.5, 0.25, 0.125]
    assert O.alpha_schedule(4, 1.0, 0.5, 0.3) == [1.0, 0.5, 0.3, 0.3]


def test_output_image_is_gauge_invariant():
    g, _, rng, _ = tiny_geometry(N=8, J=2)
    x = scaled_point(g, rng)
    rho, chat = g.unpack(x)
    a = 0.7 * np.exp(0.4j)
    x2 = g.pack(a * rho, chat / a)
    assert rel(O.coil_images(g, x2), O.coil_images(g, x)) < 1e-13
    assert rel(O.image(g, x2), O.image(g, x)) < 1e-13
