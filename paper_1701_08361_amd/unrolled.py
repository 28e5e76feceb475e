"""Unrolled, checkpointed IRGNM for differentiation (Sec. 2.2).

The same iteration as the plain solver (M Newton steps, each C CG iterations
from h = 0 on (DF^H DF + alpha_n) h = DF^H (y - F_hat(x_n)) - alpha_n (x_n -
x_prev), alpha_n = alpha_0 q^n), written with the differentiable operators of
paper_1701_08361_amd.autograd so that torch.autograd can take gradients of a
loss on the result with respect to the data y and the regularisation weight
alpha_0.  Each Newton step is checkpointed: only the iterates x_n are kept
between the forward and the backward pass, the CG iterations are recomputed.
`ops` may be an autograd.Reweighted model, which adds gradients with respect
to the Sobolev weight's parameters.

Two forms:
  "toeplitz" (default): the solver's own form.  The data enter once as the
      gridded z = F^H y (exact sum); the right-hand side is
      E_x^H (z - T E_x(rho_x, 0)) - alpha (x - x_prev) and the CG operator
      E_x^H T E_x + alpha, both through the PSF convolution T = F^H F of each
      item's turn (the PSF kernels must be in the plan).  Unknowns-space
      vectors (the iterate, h, r, p, q) are complex128 and the inner products,
      a and beta float64, as in the plain solver.  On a library plan with
      checkpointed steps the forward pass of each step is the solver's own
      Newton step (nlinv_newton_step), and the backward pass recomputes the
      step with the differentiable operators.
  "nudft": F and F^H separately through the exact non-uniform DFT (slow; the
      reference for the first form).
The CG vector algebra runs as torch operations on the device.

Newton steps and CG iterations follow the reading of the plain solver:
Re<., .> inner products, a = 0 when Re<p, q> = 0, beta = 0 when the previous
residual is 0; alpha_min = 0.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import autograd as AG


def _rdot(a, b):
    """Re<a, b> per batch item -> [B], accumulated in float64."""
    return (a.conj() * b).real.to(torch.float64).sum(dim=-1)


def _safe_div(num, den):
    zero = den == 0
    return torch.where(zero, torch.zeros_like(num), num / torch.where(zero, torch.ones_like(den), den))


def unit_start(B, R, X, device, dtype=torch.complex64):
    """(rho = 1, c = 0) for B items."""
    x = torch.zeros(B, X, dtype=dtype, device=device)
    x[:, :R * R] = 1
    return x


def _cg(apply_A, b, cg_iters):
    """C CG iterations on A h = b from h = 0 (float64 scalars)."""
    h = torch.zeros_like(b)
    r, p = b, b
    rr = _rdot(r, r)
    for _ in range(cg_iters):
        q = apply_A(p)
        a = _safe_div(rr, _rdot(p, q)).to(b.real.dtype)
        h = h + a[:, None] * p
        r = r - a[:, None] * q
        rr_new = _rdot(r, r)
        beta = _safe_div(rr_new, rr).to(b.real.dtype)
        p = r + beta[:, None] * p
        rr = rr_new
    return h


def newton_step_toeplitz(ops, turns, x, xprev, z, alpha, cg_iters, R):
    """x + h (complex128) with h from C CG iterations on the Newton system at
    x, through the PSF convolution."""
    m = AG.model(ops)
    rho_only = torch.zeros(x.shape[-1], dtype=x.real.dtype, device=x.device)
    rho_only[:R * R] = 1
    b = m.EH(x, z) - m.normal(turns, x, x * rho_only, 0.0) - alpha * (x - xprev)
    return x + _cg(lambda p: m.normal(turns, x, p, alpha), b, cg_iters)


class _LibraryStep(torch.autograd.Function):
    """One checkpointed Newton step of the Toeplitz form on a library plan.
    Forward: the solver's own Newton step (nlinv_newton_step: its kernels,
    FP64 CG; the iterate rounded to the plan's precision, complex64, as the
    solver stores it; a reweighted model runs under its coil-weight table).
    Backward: the step recomputed with the differentiable operators
    (newton_step_toeplitz) and differentiated; only the step's inputs are
    kept in between."""

    @staticmethod
    def forward(ctx, x, xprev, z, alpha, d, plan, turns, cg_iters, R, winv, alpha_value):
        ctx.plan, ctx.turns, ctx.cg_iters, ctx.R = plan, turns, cg_iters, R
        ctx.save_for_backward(x, xprev, z, alpha, d)
        dt = getattr(plan, "dtype", torch.complex64)
        xh = x.detach().to(dt, copy=True).contiguous()      # updated in place
        xp = xprev.detach().to(dt).contiguous()
        if winv is not None:
            plan.set_coil_weights(winv)
        try:
            plan.newton_step(turns, z.detach().contiguous(), xh, alpha_value, cg_iters, xp)
        finally:
            if winv is not None:
                plan.set_coil_weights(None)
        return xh.to(torch.complex128)

    @staticmethod
    def backward(ctx, g):
        saved = ctx.saved_tensors
        need = ctx.needs_input_grad[:5]
        with torch.enable_grad():
            ins = [t.detach().requires_grad_(n) if t is not None else None for t, n in zip(saved, need)]
            x, xp, z, alpha, d = ins
            m = AG.Plain(ctx.plan) if d is None else AG.Reweighted.from_diagonal(ctx.plan, ctx.R, d)
            out = newton_step_toeplitz(m, ctx.turns, x, xp, z, alpha, ctx.cg_iters, ctx.R)
            wrt = [t for t, n in zip(ins, need) if n and t is not None]
            got = iter(torch.autograd.grad(out, wrt, g, allow_unused=True)) if wrt else iter(())
        grads = [next(got) if n and t is not None else None for t, n in zip(ins, need)]
        return (*grads, None, None, None, None, None, None)


def newton_step(ops, traj, x, xprev, y, alpha, cg_iters):
    """x + h with h from C CG iterations on the Newton system at x."""
    m = AG.model(ops)
    b = m.DFH(traj, x, y - m.F(traj, x)) - alpha * (x - xprev)
    return x + _cg(lambda p: m.DFH(traj, x, m.DF(traj, x, p)) + alpha * p, b, cg_iters)


def reconstruct(ops, traj, y, R, newton=5, cg_iters=10, alpha0=1.0, alpha_q=0.5, x0=None, xprev=None,
                checkpoint_steps=True, form="toeplitz", turns=None):
    """x_M of the IRGNM for data y [B][J][S] on trajectories traj [B][K][S_r][2].
    alpha0 may be a tensor that requires grad.  form "toeplitz" needs `turns`
    (the PSF kernel of each item) and returns complex128 iterates; "nudft"
    works in the data's precision."""
    B, X = y.shape[0], ops.X
    dev = y.device
    if form == "toeplitz":
        if turns is None:
            raise ValueError("the toeplitz form needs the turns of the items' PSF kernels")
        dt = torch.complex128
        z = AG.grid(AG.model(ops).ops, traj, y)
    else:
        dt = y.dtype
    x = unit_start(B, R, X, dev, dt) if x0 is None else x0.to(dt)
    xp = unit_start(B, R, X, dev, dt) if xprev is None else xprev.to(dt)
    alpha0 = torch.as_tensor(alpha0, dtype=x.real.dtype, device=dev)
    m = AG.model(ops)
    library = form == "toeplitz" and checkpoint_steps and hasattr(m.ops, "newton_step")
    if library:
        a0 = float(alpha0.detach())
    for n in range(newton):
        alpha = alpha0 * (alpha_q ** n)
        if library:
            x = _LibraryStep.apply(x, xp, z, alpha, getattr(m, "d", None), m.ops, turns, cg_iters, R,
                                   getattr(m, "winv", None), a0 * (alpha_q ** n))
            continue
        if form == "toeplitz":
            args = (newton_step_toeplitz, ops, turns, x, xp, z, alpha, cg_iters, R)
        else:
            args = (newton_step, ops, traj, x, xp, y, alpha, cg_iters)
        x = checkpoint(*args, use_reentrant=False) if checkpoint_steps else args[0](*args[1:])
    return x


def image(ops, x, R, eps=1e-12):
    """|rho| sqrt(sum_j |c_j|^2) [B][R][R], differentiable (eps keeps the square
    root's derivative finite where every coil vanishes).  The image is formed in
    the operators' precision (complex64 for the library)."""
    x = x.to(getattr(AG.model(ops).ops, "dtype", x.dtype))
    rho = x[:, :R * R].reshape(-1, R, R)
    c = AG.model(ops).coils(x)
    return rho.abs() * torch.sqrt((c.abs() ** 2).sum(dim=1) + eps)
