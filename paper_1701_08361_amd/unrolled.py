"""Unrolled, checkpointed IRGNM for differentiation (Sec. 2.2).

The same iteration as the plain solver (M Newton steps, each C CG iterations
from h = 0 on (DF^H DF + alpha_n) h = DF^H (y - F_hat(x_n)) - alpha_n (x_n -
x_prev), alpha_n = alpha_0 q^n), written with the differentiable operators of
paper_1701_08361_amd.autograd so that torch.autograd can take gradients of a
loss on the result with respect to the data y and the regularisation weight
alpha_0.  The operators run through the C-ABI (exact non-uniform DFT, no PSF
convolution: F and F^H separately, which the adjoint rules need); the CG
vector algebra of this form runs as torch operations on the device.  Each
Newton step is checkpointed: only the iterates x_n are kept between the
forward and the backward pass, the CG iterations are recomputed.  `ops` may
be an autograd.Reweighted model, which adds gradients with respect to the
Sobolev weight's parameters.

Newton steps and CG iterations follow the reading of the plain solver:
Re<., .> inner products, a = 0 when Re<p, q> = 0, beta = 0 when the previous
residual is 0; alpha_min = 0.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import autograd as AG


def _rdot(a, b):
    """Re<a, b> per batch item -> [B]."""
    return (a.conj() * b).real.sum(dim=-1)


def _safe_div(num, den):
    zero = den == 0
    return torch.where(zero, torch.zeros_like(num), num / torch.where(zero, torch.ones_like(den), den))


def unit_start(B, R, X, device, dtype=torch.complex64):
    """(rho = 1, c = 0) for B items."""
    x = torch.zeros(B, X, dtype=dtype, device=device)
    x[:, :R * R] = 1
    return x


def newton_step(ops, traj, x, xprev, y, alpha, cg_iters):
    """x + h with h from C CG iterations on the Newton system at x."""
    m = AG.model(ops)
    b = m.DFH(traj, x, y - m.F(traj, x)) - alpha * (x - xprev)
    h = torch.zeros_like(b)
    r, p = b, b
    rr = _rdot(r, r)
    for _ in range(cg_iters):
        q = m.DFH(traj, x, m.DF(traj, x, p)) + alpha * p
        a = _safe_div(rr, _rdot(p, q))
        h = h + a[:, None] * p
        r = r - a[:, None] * q
        rr_new = _rdot(r, r)
        beta = _safe_div(rr_new, rr)
        p = r + beta[:, None] * p
        rr = rr_new
    return x + h


def reconstruct(ops, traj, y, R, newton=5, cg_iters=10, alpha0=1.0, alpha_q=0.5, x0=None, xprev=None,
                checkpoint_steps=True):
    """x_M of the IRGNM for data y [B][J][S] on trajectories traj [B][K][S_r][2].
    alpha0 may be a tensor that requires grad."""
    B, X = y.shape[0], ops.X
    dev, dt = y.device, y.dtype
    x = unit_start(B, R, X, dev, dt) if x0 is None else x0
    xp = unit_start(B, R, X, dev, dt) if xprev is None else xprev
    alpha0 = torch.as_tensor(alpha0, dtype=y.real.dtype, device=dev)
    for n in range(newton):
        alpha = alpha0 * (alpha_q ** n)
        if checkpoint_steps:
            x = checkpoint(newton_step, ops, traj, x, xp, y, alpha, cg_iters, use_reentrant=False)
        else:
            x = newton_step(ops, traj, x, xp, y, alpha, cg_iters)
    return x


def image(ops, x, R, eps=1e-12):
    """|rho| sqrt(sum_j |c_j|^2) [B][R][R], differentiable (eps keeps the square
    root's derivative finite where every coil vanishes)."""
    rho = x[:, :R * R].reshape(-1, R, R)
    c = AG.model(ops).coils(x)
    return rho.abs() * torch.sqrt((c.abs() ** 2).sum(dim=1) + eps)
