"""torch.autograd form of the NLINV operators (Sec. 2.2).

F_hat(x) = F(rho . W^-1 c_hat_j), its derivative DF_x(dx) and the adjoint
DF_x^H(dy) as differentiable functions whose backward passes are the
hand-written adjoints of the C-ABI (nlinv_apply_DF / nlinv_apply_DFH).  No
arithmetic happens here: every forward and backward step is one library call.

The gradient rules follow from two facts of the model:
  * F_hat is bilinear in (rho, c_hat) with no conjugation, so for a real loss
    the gradient through y = F_hat(x) is DF_x^H(g);
  * DF_x(dx) is symmetric in its two arguments, DF_x(dx) = DF_dx(x), so its
    gradient with respect to x is DF_dx^H(g), and by the adjoint identity the
    gradient of DF_x^H(dy) with respect to x is DF_g^H(dy).
Gradients use PyTorch's convention for complex tensors: for a real loss L,
dL = Re<grad, dx>.

`ops` is any object with apply_F / apply_DF / apply_DFH(traj, xhat, ...),
coils(xhat, want_img=False) and apply_WH(coils) in the shapes of
paper_1701_08361_amd.nlinv.Plan (xhat [B][X], data [B][J][S], coil images
[B][J][R][R]); the PSF-convolution form below also uses grid, nudft,
apply_normal2, apply_E and apply_EH.  Reweighted gives the same operators under another Sobolev
weight, differentiable in its parameters.
"""
from __future__ import annotations

import math

import torch


class _F(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xhat, ops, traj):
        ctx.ops, ctx.traj = ops, traj
        ctx.save_for_backward(xhat)
        return ops.apply_F(traj, xhat.contiguous())

    @staticmethod
    def backward(ctx, g):
        (xhat,) = ctx.saved_tensors
        gx = ctx.ops.apply_DFH(ctx.traj, xhat.contiguous(), g.contiguous()) if ctx.needs_input_grad[0] else None
        return gx, None, None


class _DF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xhat, dx, ops, traj):
        ctx.ops, ctx.traj = ops, traj
        ctx.save_for_backward(xhat, dx)
        return ops.apply_DF(traj, xhat.contiguous(), dx.contiguous())

    @staticmethod
    def backward(ctx, g):
        xhat, dx = ctx.saved_tensors
        g = g.contiguous()
        gx = ctx.ops.apply_DFH(ctx.traj, dx.contiguous(), g) if ctx.needs_input_grad[0] else None
        gdx = ctx.ops.apply_DFH(ctx.traj, xhat.contiguous(), g) if ctx.needs_input_grad[1] else None
        return gx, gdx, None, None


class _DFH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xhat, dy, ops, traj):
        ctx.ops, ctx.traj = ops, traj
        ctx.save_for_backward(xhat, dy)
        return ops.apply_DFH(traj, xhat.contiguous(), dy.contiguous())

    @staticmethod
    def backward(ctx, g):
        xhat, dy = ctx.saved_tensors
        g = g.contiguous()
        gx = ctx.ops.apply_DFH(ctx.traj, g, dy.contiguous()) if ctx.needs_input_grad[0] else None
        gdy = ctx.ops.apply_DF(ctx.traj, xhat.contiguous(), g) if ctx.needs_input_grad[1] else None
        return gx, gdy, None, None


class _Coils(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xhat, ops):
        ctx.ops = ops
        c, _ = ops.coils(xhat.contiguous(), want_img=False)
        return c

    @staticmethod
    def backward(ctx, g):
        return ctx.ops.apply_WH(g.contiguous()), None


def coils(ops, xhat):
    """Coil images c_j = W^-1 c_hat_j [B][J][R][R] (linear in the coil block)."""
    return _Coils.apply(xhat, ops)


# ---------------------------------------------------------------------------
# The PSF-convolution (Toeplitz) form.  With E_x the image-space part of the
# derivative (DF_x = F E_x, E_x(p)_j = c_j d_rho + rho W^-1 d_c_hat_j) and
# T = F^H F, the Newton right-hand side is E_x^H (z - T E_x(rho_x, 0)) with
# z = F^H y, and the CG operator is E_x^H T E_x + alpha.  E_x(p) is
# symmetric bilinear in (x, p), so for a real loss with upstream gradient g:
#   z = F^H y              : grad_y = F g
#   v = E_x^H img          : grad_img = E_x g,  grad_x = E_g^H img
#   q = E_x^H T E_x p + a p: grad_p = E_x^H T E_x g + a g,
#                            grad_x = E_g^H T E_x p + E_p^H T E_x g,
#                            grad_a = Re<p, g>
# Unknowns-space vectors are complex128; linearisation points are rounded to
# the operators' precision (`ops.dtype`: complex64 for the library, whose
# solver stores its iterates so too).
# ---------------------------------------------------------------------------

def _pt(ops, t):
    return t.detach().to(getattr(ops, "dtype", torch.complex64)).contiguous()


class _Grid(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, ops, traj):
        ctx.ops, ctx.traj = ops, traj
        return ops.grid(traj, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.ops.nudft(ctx.traj, g.contiguous()), None, None


class _EH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, img, ops):
        ctx.ops = ops
        ctx.save_for_backward(x, img)
        return ops.apply_EH(_pt(ops, x), img.contiguous())

    @staticmethod
    def backward(ctx, g):
        x, img = ctx.saved_tensors
        g = g.contiguous()
        gx = ctx.ops.apply_EH(_pt(ctx.ops, g), img.contiguous()) if ctx.needs_input_grad[0] else None
        gimg = ctx.ops.apply_E(_pt(ctx.ops, x), g) if ctx.needs_input_grad[1] else None
        return gx, gimg, None


class _Normal(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, p, alpha, ops, turns):
        ctx.ops, ctx.turns = ops, turns
        ctx.save_for_backward(x, p, alpha)
        xc = _pt(ops, x)
        return ops.apply_normal2(turns, xc, xc, p.contiguous(), float(alpha))

    @staticmethod
    def backward(ctx, g):
        x, p, alpha = ctx.saved_tensors
        ops, turns = ctx.ops, ctx.turns
        g = g.contiguous()
        xc = _pt(ops, x)
        gx = gp = ga = None
        if ctx.needs_input_grad[0]:
            gx = (ops.apply_normal2(turns, _pt(ops, g), xc, p.contiguous(), 0.0)
                  + ops.apply_normal2(turns, _pt(ops, p), xc, g, 0.0))
        if ctx.needs_input_grad[1]:
            gp = ops.apply_normal2(turns, xc, xc, g, float(alpha))
        if ctx.needs_input_grad[2]:
            ga = (p.conj() * g).real.sum().to(alpha.dtype)
        return gx, gp, ga, None, None


def grid(ops, traj, y):
    """z = F^H y [B][J][R][R] (exact sum), differentiable in y."""
    return _Grid.apply(y, ops, traj)


def EH(ops, x, img):
    """E_x^H img [B][X] complex128, differentiable in x (complex128) and img."""
    return _EH.apply(x, img, ops)


def normal(ops, turns, x, p, alpha):
    """E_x^H T E_x p + alpha p [B][X] complex128, differentiable in x, p and alpha."""
    return _Normal.apply(x, p, torch.as_tensor(alpha, dtype=torch.float64, device=p.device), ops, turns)


class Reweighted:
    """The operators of the model under another Sobolev weight
    w'(k) = (1 + a |k|^2)^l (Sec. 3.2, Fig. weight_func), differentiable in a
    and l, built from operators `ops` of the reference weight
    w(k) = (1 + a_ref |k|^2)^l_ref.

    The coil synthesis divides the coil spectrum by the weight before the
    inverse transform, so W'^-1 c_hat = W^-1 (c_hat . w / w'): with the real
    diagonal D = diag(1 on rho, w / w' on every coil block),
        F'(x) = F(D x),  DF'_x(dx) = DF_{D x}(D dx),  DF'^H_x(dy) = D DF^H_{D x}(dy),
        coils'(x) = coils(D x).
    D is formed here from a and l (tensors that may require grad) on the
    centred G_c x G_c spectrum, k = kappa / G, in the layout of x_hat; the
    operator calls themselves go through the autograd functions above.
    """

    def __init__(self, ops, G, Gc, R, J, a, l, a_ref=880.0, l_ref=16.0):
        self.ops, self.X, self.R = ops, ops.X, R
        dev = a.device if torch.is_tensor(a) else None
        kap = (torch.arange(Gc, dtype=torch.float64, device=dev) - Gc // 2) / G
        k2 = kap[:, None] ** 2 + kap[None, :] ** 2
        a = torch.as_tensor(a, dtype=torch.float64, device=dev)
        l = torch.as_tensor(l, dtype=torch.float64, device=dev)
        # w / w' in logarithms: the weights themselves reach 1e23 at the spectrum's corners
        ratio = torch.exp(l_ref * torch.log1p(a_ref * k2) - l * torch.log1p(a * k2))
        self.d = torch.cat([torch.ones(R * R, dtype=torch.float64, device=dev), ratio.reshape(-1).repeat(J)])
        # the coil-weight table 1 / (G w') of this weight, for solvers that take one (no gradient)
        with torch.no_grad():
            self.winv = torch.exp(-math.log(G) - l * torch.log1p(a * k2))

    @classmethod
    def from_diagonal(cls, ops, R, d):
        """The model of the diagonal d itself (no weight parameters)."""
        m = cls.__new__(cls)
        m.ops, m.X, m.R, m.d, m.winv = ops, ops.X, R, d, None
        return m

    def _scale(self, x):
        return x * self.d.to(device=x.device, dtype=x.real.dtype)

    def F(self, traj, xhat):
        return F(self.ops, traj, self._scale(xhat))

    def DF(self, traj, xhat, dx):
        return DF(self.ops, traj, self._scale(xhat), self._scale(dx))

    def DFH(self, traj, xhat, dy):
        return self._scale(DFH(self.ops, traj, self._scale(xhat), dy))

    def coils(self, xhat):
        return coils(self.ops, self._scale(xhat))

    def normal(self, turns, x, p, alpha):
        # N' = D N_{D x} D + alpha (the weight ratio D is real)
        return self._scale(normal(self.ops, turns, self._scale(x), self._scale(p), 0.0)) + alpha * p

    def EH(self, x, img):
        return self._scale(EH(self.ops, self._scale(x), img))


class Plain:
    """The operators of `ops` in the interface of Reweighted."""

    def __init__(self, ops):
        self.ops, self.X = ops, ops.X

    def F(self, traj, xhat):
        return F(self.ops, traj, xhat)

    def DF(self, traj, xhat, dx):
        return DF(self.ops, traj, xhat, dx)

    def DFH(self, traj, xhat, dy):
        return DFH(self.ops, traj, xhat, dy)

    def coils(self, xhat):
        return coils(self.ops, xhat)

    def normal(self, turns, x, p, alpha):
        return normal(self.ops, turns, x, p, alpha)

    def EH(self, x, img):
        return EH(self.ops, x, img)


def model(ops):
    """Reweighted / Plain models pass through; raw operators are wrapped."""
    return ops if isinstance(ops, (Reweighted, Plain)) else Plain(ops)


def F(ops, traj, xhat):
    """y = F_hat(xhat) [B][J][S], differentiable in xhat."""
    return _F.apply(xhat, ops, traj)


def DF(ops, traj, xhat, dx):
    """DF_xhat(dx) [B][J][S], differentiable in xhat and dx."""
    return _DF.apply(xhat, dx, ops, traj)


def DFH(ops, traj, xhat, dy):
    """DF_xhat^H(dy) [B][X], differentiable in xhat and dy."""
    return _DFH.apply(xhat, dy, ops, traj)
