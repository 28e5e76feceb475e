"""FP64 CPU oracle for the NLINV hot path (Schaetz, Voit, Frahm, Uecker,
"Accelerated Computing in MRI: Real-Time Imaging Using Non-Linear Inverse
Reconstruction").

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path
(the HIP library and its binding) never calls it, and this module imports
nothing from the product path; the only shared code is the seeded input
generator, which holds no reconstruction arithmetic.

Everything is plain NumPy in complex128/float64 and follows the paper's
definitions literally:
  * every uniform Fourier transform is a dense DFT matrix (no FFT),
  * the non-uniform transform is the exact non-uniform DFT sum,
  * pad / crop are explicit zero-filling / slicing of centred arrays,
  * the normal operator is evaluated through the point-spread-function
    convolution (Sec. 2.2 and its footnote) and, for checking, through the
    explicit non-uniform DFT and its adjoint,
  * IRGNM + CG run with fixed iteration counts.

Readings of points the paper leaves open (all shared with the HIP path):
  - F_u is the unitary 2D DFT on the G x G grid, centred index sets
    [-floor(n/2), ceil(n/2)-1]; the PSF kernel P is the unnormalised DFT of
    the PSF so that F_u^-1 (P . F_u v) is the cyclic convolution psf * v.
  - Image pixels sit at integer coordinates r in [-R/2, R/2)^2, R = G/2;
    the non-uniform DFT uses exp(-i 2 pi k.r) with k in cycles/pixel and
    the unitary scale 1/R (the same normalisation as F_u: F is unitary when
    the samples are the R x R Cartesian frequencies of the field of view).
    Without it the data term of every Newton system is R^2 times heavier
    than alpha_n and CG becomes too ill-conditioned for float32.
  - The PSF is kept on lags |d_x|,|d_y| <= R-1 (the only lags a difference
    of two FOV pixels can take); all other lags of the G-grid are zero,
    which makes P real.
  - Sobolev weight w(k) = (1 + 880 |k|^2)^16 with k = kappa/G (Sec. 3.2,
    Fig. weight_func); W multiplies the coil spectra by w and leaves the
    image untouched (Sec. 2.2), so in the variables x_hat = W x the coil
    block holds c_hat_j = w . F_u(pad c_j) restricted to the G_c x G_c
    centre, G_c = floor(G/4) (Sec. 3.2, coil cropping).
  - IRGNM schedule alpha_0 = 1, alpha_{n+1} = max(alpha_n * 0.5, alpha_min);
    CG from h = 0 with C iterations, real part of the inner products,
    a = 0 when Re<p, q> = 0 and beta = 0 when the previous residual is 0.
  - Output image |rho| * sqrt(sum_j |c_j|^2).

Vector layout of x_hat (length R*R + J*G_c*G_c): the image rho as R x R
row-major [y, x], followed by the J coil spectra, each G_c x G_c row-major
[kappa_y, kappa_x] with DC at index (G_c//2, G_c//2).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# ---------------------------------------------------------------------------
# sizes and index sets
# ---------------------------------------------------------------------------


def sizes(N: int, G: int | None = None):
    """Grid sizes (Sec. 3.2): G = 2 gamma N (gamma = 1 unless G is given),
    reconstructed side R = G/2, coil-spectrum side G_c = floor(G/4)."""
    G = 2 * N if G is None else int(G)
    if G % 2:
        raise ValueError("G must be even")
    R = G // 2
    if R < N:
        raise ValueError("G must be at least 2N")
    Gc = G // 4
    return R, G, Gc


def centred(n: int) -> np.ndarray:
    """Centred index set [-floor(n/2), ceil(n/2) - 1]."""
    return np.arange(n) - n // 2


def pad(a: np.ndarray, G: int) -> np.ndarray:
    """Zero-fill the trailing n x n block(s) of `a` into the centre of G x G."""
    n = a.shape[-1]
    out = np.zeros(a.shape[:-2] + (G, G), dtype=np.complex128)
    o = G // 2 - n // 2
    out[..., o:o + n, o:o + n] = a
    return out


def crop(a: np.ndarray, n: int) -> np.ndarray:
    """Centre n x n block of the trailing G x G dimensions."""
    G = a.shape[-1]
    o = G // 2 - n // 2
    return a[..., o:o + n, o:o + n]


# ---------------------------------------------------------------------------
# dense uniform DFT
# ---------------------------------------------------------------------------

def dft_matrix(G: int, sign: int = -1) -> np.ndarray:
    """Unitary 1D DFT matrix on the centred index set: exp(sign i 2 pi k n / G)/sqrt(G)."""
    n = centred(G).astype(np.float64)
    return np.exp(sign * 2j * np.pi * np.outer(n, n) / G) / np.sqrt(G)


def fft2u(a: np.ndarray) -> np.ndarray:
    """Unitary forward 2D DFT F_u of the trailing G x G dims (dense matrices)."""
    D = dft_matrix(a.shape[-1], -1)
    return D @ a @ D.T


def ifft2u(a: np.ndarray) -> np.ndarray:
    """Unitary inverse 2D DFT F_u^-1 of the trailing G x G dims."""
    D = dft_matrix(a.shape[-1], +1)
    return D @ a @ D.T


# ---------------------------------------------------------------------------
# Sobolev weighting W (Sec. 2.2; weight of Fig. weight_func)
# ---------------------------------------------------------------------------

def sobolev_weight(G: int, Gc: int, a: float = 880.0, l: float = 16.0) -> np.ndarray:
    """w(kappa) = (1 + a |kappa/G|^2)^l on the centred G_c x G_c coil spectrum."""
    k = centred(Gc).astype(np.float64) / G
    return (1.0 + a * (k[:, None] ** 2 + k[None, :] ** 2)) ** l


def winv(chat: np.ndarray, G: int, R: int, w: np.ndarray) -> np.ndarray:
    """W^-1: coil spectra [..., Gc, Gc] -> coil images [..., R, R]:
    crop_R F_u^-1 pad_G (chat / w)."""
    return crop(ifft2u(pad(chat / w, G)), R)


def winvh(v: np.ndarray, G: int, Gc: int, w: np.ndarray) -> np.ndarray:
    """W^-H, the adjoint of W^-1: images [..., R, R] -> spectra [..., Gc, Gc]:
    (1/w) . crop_Gc F_u pad_G v."""
    return crop(fft2u(pad(v, G)), Gc) / w


# ---------------------------------------------------------------------------
# non-uniform DFT (the operator called script-F in Sec. 2.2)
# ---------------------------------------------------------------------------

def _phase_factors(traj: np.ndarray, R: int, sign: int):
    k = np.asarray(traj, dtype=np.float64).reshape(-1, 2)
    c = centred(R).astype(np.float64)
    ex = np.exp(sign * 2j * np.pi * np.outer(k[:, 0], c))     # [S, R] over x
    ey = np.exp(sign * 2j * np.pi * np.outer(k[:, 1], c))     # [S, R] over y
    return ex, ey


def nudft(u: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """(F u)_s = (1/R) sum_r u(r) exp(-i 2 pi k_s.r): images [..., R, R] -> [..., S].
    Evaluated exactly; the sum over r is split into its x and y parts."""
    R = u.shape[-1]
    ex, ey = _phase_factors(traj, R, -1)
    a = u @ ex.T                                   # [..., y, s] = sum_x u[y,x] ex[s,x]
    return np.einsum("sy,...ys->...s", ey, a) / R


def nudft_adjoint(v: np.ndarray, traj: np.ndarray, R: int) -> np.ndarray:
    """(F^H v)(r) = (1/R) sum_s v_s exp(+i 2 pi k_s.r): [..., S] -> [..., R, R]."""
    ex, ey = _phase_factors(traj, R, +1)
    v = np.asarray(v, dtype=np.complex128)
    return np.matmul(ey.T * v[..., None, :], ex) / R   # [..., y, s] @ [s, x]


def nudft_matrix(traj: np.ndarray, R: int) -> np.ndarray:
    """Dense S x R^2 matrix of the non-uniform DFT (row-major pixel order)."""
    k = np.asarray(traj, dtype=np.float64).reshape(-1, 2)
    c = centred(R).astype(np.float64)
    Y, X = np.meshgrid(c, c, indexing="ij")
    return np.exp(-2j * np.pi * (np.outer(k[:, 0], X.ravel()) + np.outer(k[:, 1], Y.ravel()))) / R


# ---------------------------------------------------------------------------
# gridding and the PSF convolution (Sec. 2.2 footnote, Sec. 3.1)
# ---------------------------------------------------------------------------

def grid(y: np.ndarray, traj: np.ndarray, R: int) -> np.ndarray:
    """Gridded data z_j = F^H y_j on the R x R field of view: [J, S] -> [J, R, R]."""
    return nudft_adjoint(np.asarray(y, dtype=np.complex128), traj, R)


def psf_lags(traj: np.ndarray, R: int) -> np.ndarray:
    """psf(d) = (1/R^2) sum_s exp(+i 2 pi k_s.d) for lags d in [-(R-1), R-1]^2
    -> [2R-1, 2R-1] [dy, dx], so that (F^H F u)(r) = sum_r' psf(r - r') u(r')."""
    k = np.asarray(traj, dtype=np.float64).reshape(-1, 2)
    d = np.arange(-(R - 1), R).astype(np.float64)
    ex = np.exp(2j * np.pi * np.outer(k[:, 0], d))
    ey = np.exp(2j * np.pi * np.outer(k[:, 1], d))
    return (ey.T @ ex) / (R * R)


def psf_kernel(traj: np.ndarray, R: int, G: int, keep_imag: bool = False) -> np.ndarray:
    """P = unnormalised 2D DFT (on the centred G-grid) of the PSF embedded at its
    lags, all other lags zero.  Real up to rounding; the real part is returned."""
    if G < 2 * R - 1:
        raise ValueError("the PSF convolution needs G >= 2R - 1")
    psf = np.zeros((G, G), dtype=np.complex128)
    o = G // 2 - (R - 1)
    psf[o:o + 2 * R - 1, o:o + 2 * R - 1] = psf_lags(traj, R)
    P = G * fft2u(psf)
    return P if keep_imag else P.real


def toeplitz(u: np.ndarray, P: np.ndarray) -> np.ndarray:
    """T u = crop_R F_u^-1 (P . F_u pad_G u)  (equals F^H F u exactly)."""
    G = P.shape[-1]
    R = u.shape[-1]
    return crop(ifft2u(P * fft2u(pad(u, G))), R)


# ---------------------------------------------------------------------------
# the NLINV operators in the variables x_hat = (rho, c_hat)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Geometry:
    R: int
    G: int
    Gc: int
    J: int
    w: np.ndarray            # Sobolev weight on the Gc x Gc coil spectrum

    @property
    def X(self) -> int:
        return self.R * self.R + self.J * self.Gc * self.Gc

    @classmethod
    def make(cls, N: int, J: int, G: int | None = None, a: float = 880.0, l: float = 16.0):
        R, G, Gc = sizes(N, G)
        return cls(R=R, G=G, Gc=Gc, J=J, w=sobolev_weight(G, Gc, a, l))

    def unpack(self, x: np.ndarray):
        x = np.asarray(x, dtype=np.complex128)
        rho = x[:self.R * self.R].reshape(self.R, self.R)
        chat = x[self.R * self.R:].reshape(self.J, self.Gc, self.Gc)
        return rho, chat

    def pack(self, rho: np.ndarray, chat: np.ndarray) -> np.ndarray:
        return np.concatenate([np.ravel(rho), np.ravel(chat)]).astype(np.complex128)

    def initial(self) -> np.ndarray:
        """First frame: rho = 1, c = 0 (Sec. 3.3, temporal decomposition)."""
        return self.pack(np.ones((self.R, self.R)), np.zeros((self.J, self.Gc, self.Gc)))

    def coils(self, x: np.ndarray) -> np.ndarray:
        """c_j = W^-1 c_hat_j -> [J, R, R]."""
        _, chat = self.unpack(x)
        return winv(chat, self.G, self.R, self.w)


def F_hat(g: Geometry, x: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """F_hat(x_hat)_j = F(rho . W^-1 c_hat_j) -> [J, S]  (F = F o C, x = W^-1 x_hat)."""
    rho, _ = g.unpack(x)
    return nudft(rho[None] * g.coils(x), traj)


def DF_hat(g: Geometry, x: np.ndarray, dx: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """Derivative at x_hat: DF(d rho, d c_hat)_j = F(c_j d rho + rho W^-1 d c_hat_j)."""
    rho, _ = g.unpack(x)
    c = g.coils(x)
    drho, dchat = g.unpack(dx)
    dc = winv(dchat, g.G, g.R, g.w)
    return nudft(c * drho[None] + rho[None] * dc, traj)


def image_adjoint(g: Geometry, x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The image-space part of DF^H (normal-operator equation, Sec. 2.2):
    t [J, R, R] -> (sum_j conj(c_j) t_j ; W^-H (conj(rho) t_j))."""
    rho, _ = g.unpack(x)
    c = g.coils(x)
    top = np.sum(np.conj(c) * t, axis=0)
    bottom = winvh(np.conj(rho)[None] * t, g.G, g.Gc, g.w)
    return g.pack(top, bottom)


def DFH_hat(g: Geometry, x: np.ndarray, v: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """Adjoint derivative: DF^H v = image_adjoint(F^H v_j) for radial samples v [J, S]."""
    return image_adjoint(g, x, nudft_adjoint(np.asarray(v, np.complex128), traj, g.R))


def normal(g: Geometry, x: np.ndarray, dx: np.ndarray, P: np.ndarray) -> np.ndarray:
    """DF^H DF dx with t_j = T(c_j d rho + rho W^-1 d c_hat_j) through the PSF kernel P."""
    rho, _ = g.unpack(x)
    c = g.coils(x)
    drho, dchat = g.unpack(dx)
    u = c * drho[None] + rho[None] * winv(dchat, g.G, g.R, g.w)
    return image_adjoint(g, x, toeplitz(u, P))


def normal_explicit(g: Geometry, x: np.ndarray, dx: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """The same operator as DF^H(DF(dx)) through the non-uniform DFT."""
    return DFH_hat(g, x, DF_hat(g, x, dx, traj), traj)


# ---------------------------------------------------------------------------
# IRGNM with CG (Sec. 2.2)
# ---------------------------------------------------------------------------

def rdot(a: np.ndarray, b: np.ndarray) -> float:
    """Real part of the Euclidean inner product <a, b> = sum conj(a) b."""
    return float(np.real(np.vdot(a, b)))


def cg(apply_A, b: np.ndarray, iters: int) -> np.ndarray:
    """Conjugate gradients for A h = b from h = 0, a fixed number of iterations."""
    h = np.zeros_like(b)
    r = b.copy()
    p = b.copy()
    rr = rdot(r, r)
    for _ in range(iters):
        q = apply_A(p)
        pq = rdot(p, q)
        a = rr / pq if pq != 0.0 else 0.0
        h = h + a * p
        r = r - a * q
        rr_new = rdot(r, r)
        beta = rr_new / rr if rr != 0.0 else 0.0
        p = r + beta * p
        rr = rr_new
    return h


def alpha_schedule(M: int, alpha0: float = 1.0, q: float = 0.5, alpha_min: float = 0.0):
    out, a = [], float(alpha0)
    for _ in range(M):
        out.append(a)
        a = max(a * q, alpha_min)
    return out


def newton_rhs(g: Geometry, x: np.ndarray, xprev: np.ndarray, z: np.ndarray, P: np.ndarray,
               alpha: float) -> np.ndarray:
    """Right-hand side of the IRGNM update: DF^H (y - F_hat x_n) - alpha_n (x_n - x_prev),
    with DF^H (y - F_hat x_n) formed in image space as image_adjoint(z_j - T(rho c_j))."""
    rho, _ = g.unpack(x)
    c = g.coils(x)
    r = np.asarray(z, np.complex128) - toeplitz(rho[None] * c, P)
    return image_adjoint(g, x, r) - alpha * (np.asarray(x) - np.asarray(xprev))


def newton_step(g: Geometry, x: np.ndarray, xprev: np.ndarray, z: np.ndarray, P: np.ndarray,
                alpha: float, cg_iters: int) -> np.ndarray:
    """One IRGNM step: solve (DF^H DF + alpha I) h = rhs by CG; return h."""
    b = newton_rhs(g, x, xprev, z, P, alpha)
    return cg(lambda p: normal(g, x, p, P) + alpha * p, b, cg_iters)


def reconstruct(g: Geometry, z: np.ndarray, P: np.ndarray, xprev: np.ndarray | None = None,
                x0: np.ndarray | None = None, newton: int = 7, cg_iters: int = 10,
                alpha0: float = 1.0, alpha_q: float = 0.5, alpha_min: float = 0.0,
                trace: list | None = None) -> np.ndarray:
    """IRGNM: x_{n+1} = x_n + h_n for n = 0..M-1 (fixed counts)."""
    x = g.initial() if x0 is None else np.asarray(x0, np.complex128).copy()
    xp = g.initial() if xprev is None else np.asarray(xprev, np.complex128)
    for alpha in alpha_schedule(newton, alpha0, alpha_q, alpha_min):
        h = newton_step(g, x, xp, z, P, alpha, cg_iters)
        if trace is not None:
            trace.append(h.copy())
        x = x + h
    return x


def image(g: Geometry, x: np.ndarray) -> np.ndarray:
    """Combined image |rho| sqrt(sum_j |c_j|^2)  -> [R, R] float64."""
    rho, _ = g.unpack(x)
    c = g.coils(x)
    return np.abs(rho) * np.sqrt(np.sum(np.abs(c) ** 2, axis=0))


def coil_images(g: Geometry, x: np.ndarray) -> np.ndarray:
    """rho . c_j -> [J, R, R] (invariant under rho -> a rho, c -> c / a)."""
    rho, _ = g.unpack(x)
    return rho[None] * g.coils(x)


# ---------------------------------------------------------------------------
# frame series: strict order and relaxed temporal coupling (Sec. 3.3,
# temporal decomposition, equation for h(n, m))
# ---------------------------------------------------------------------------

def relaxed_sources(F: int, l: int, o: int) -> list:
    """Source frame s(n) of every frame n < F for the Newton steps m < M-1.

    The equation for h(n, m) sends frame n to frame n-1 for n <= l, and for
    n > l to the most recent finished frame in [n-o, n-1].  Reading of
    "most recent finished": frames after l are taken in consecutive groups of
    o frames, l+1 .. l+o, l+o+1 .. l+2o, ...; a group starts once the frame
    before it has finished, so that frame is the most recent finished one
    for every member of the group (it lies in [n-o, n-1]).  Frame 0 has no
    source (-1: rho = 1, c = 0)."""
    if F < 0 or l < 0 or o < 1:
        raise ValueError("need F >= 0, l >= 0, o >= 1")
    src = []
    for n in range(F):
        if n == 0:
            src.append(-1)
        elif n <= l:
            src.append(n - 1)
        else:
            start = l + 1 + ((n - l - 1) // o) * o
            src.append(start - 1)
    return src


def reconstruct_series(g: Geometry, zs, Ps, sources: list | None = None, newton: int = 7,
                       cg_iters: int = 10, alpha0: float = 1.0, alpha_q: float = 0.5,
                       alpha_min: float = 0.0) -> list:
    """Reconstruct frames n = 0 .. F-1 of one series (zs[n]: gridded data,
    Ps[n]: PSF kernel of the frame's turn).

    Frame n starts from x_{h(n, 0)} and Newton step m is regularised towards
    x_{h(n, m)}, where h(n, m) = n - 1 for the last step m = M-1 and
    h(n, m) = sources[n] for m < M-1 (equation for h(n, m), Sec. 3.3).
    sources = None is the strict order h(n, m) = n - 1.  Frame 0 starts from
    and is regularised towards (rho = 1, c = 0) (Sec. 3.3)."""
    F = len(zs)
    if sources is None:
        sources = [n - 1 for n in range(F)]
    alphas = alpha_schedule(newton, alpha0, alpha_q, alpha_min)
    out: list = []

    def frame(k: int) -> np.ndarray:
        return g.initial() if k < 0 else out[k]

    for n in range(F):
        h = [n - 1 if m == newton - 1 else sources[n] for m in range(newton)]
        if n == 0:
            h = [-1] * newton
        x = frame(h[0]).copy()
        for m, alpha in enumerate(alphas):
            x = x + newton_step(g, x, frame(h[m]), zs[n], Ps[n], alpha, cg_iters)
        out.append(x)
    return out


# ---------------------------------------------------------------------------
# channel compression (Sec. 3.1, preprocessing, with its calibration phase)
# ---------------------------------------------------------------------------

def compression_matrix(y0: np.ndarray, J: int) -> np.ndarray:
    """Compression transform [J, J_phys] from a calibration frame y0 [J_phys, S].
    Reading (the paper names channel compression and its calibration phase but
    no method): principal components; the rows are the conjugated eigenvectors
    of the channel covariance y0 y0^H for its J largest eigenvalues, in
    descending order (each row fixed only up to a phase)."""
    y0 = np.asarray(y0, np.complex128)
    cov = y0 @ y0.conj().T
    w, V = np.linalg.eigh(cov)
    order = np.argsort(w)[::-1][:J]
    return V[:, order].conj().T


def compress(cc: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Virtual channels y_v[j] = sum_p cc[j, p] y[p]: [J, J_phys] x [..., J_phys, S]."""
    return np.asarray(cc, np.complex128) @ np.asarray(y, np.complex128)
