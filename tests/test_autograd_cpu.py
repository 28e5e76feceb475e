"""The autograd form of F_hat, DF and DF^H (paper_1701_08361_amd.autograd),
checked on the CPU by torch.autograd.gradcheck in complex128 with the FP64
oracle standing in for the HIP operators: this pins the gradient rules of the
wrappers (which adjoint, at which linearisation point) independently of the
GPU, which the GPU tests then run with the C-ABI operators."""
import numpy as np
import pytest
import torch

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import autograd as AG
from paper_1701_08361_amd import synth


class OracleOps:
    """apply_F / apply_DF / apply_DFH in the shapes of the C-ABI binding, FP64."""

    def __init__(self, g):
        self.g = g

    def _each(self, fn, *args):
        out = [fn(*[a[b].detach().numpy() for a in args]) for b in range(args[0].shape[0])]
        return torch.from_numpy(np.stack(out))

    def apply_F(self, traj, xhat):
        return self._each(lambda t, x: O.F_hat(self.g, x, t).reshape(self.g.J, -1), traj, xhat)

    def apply_DF(self, traj, xhat, dx):
        return self._each(lambda t, x, d: O.DF_hat(self.g, x, d, t).reshape(self.g.J, -1), traj, xhat, dx)

    def apply_DFH(self, traj, xhat, dy):
        return self._each(lambda t, x, v: O.DFH_hat(self.g, x, v, t), traj, xhat, dy)


def _setup(B=2, N=8, J=2, K=3, seed=0):
    g = O.Geometry.make(N, J)
    traj = torch.from_numpy(np.stack([synth.radial_trajectory(N, K, 2 * N, b, B) for b in range(B)]).astype(np.float64))
    rng = np.random.default_rng(seed)
    cx = lambda *s: torch.from_numpy(rng.standard_normal(s) + 1j * rng.standard_normal(s))
    return OracleOps(g), traj, g, cx


def test_F_gradcheck():
    ops, traj, g, cx = _setup()
    x = cx(2, g.X).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: AG.F(ops, traj, x), (x,), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_DF_gradcheck():
    ops, traj, g, cx = _setup(seed=1)
    x = cx(2, g.X).requires_grad_(True)
    dx = cx(2, g.X).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x, d: AG.DF(ops, traj, x, d), (x, dx), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)


def test_DFH_gradcheck():
    ops, traj, g, cx = _setup(seed=2)
    S = traj.shape[1] * traj.shape[2]
    x = cx(2, g.X).requires_grad_(True)
    dy = cx(2, g.J, S).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x, v: AG.DFH(ops, traj, x, v), (x, dy), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)


def test_data_fidelity_gradient_is_the_gauss_newton_rhs():
    """grad of ||F(x) - y||^2 = 2 DF_x^H (F(x) - y): the right-hand side of the
    IRGNM update (without regularisation) up to the factor -2."""
    ops, traj, g, cx = _setup(B=1, seed=3)
    x = cx(1, g.X).requires_grad_(True)
    y = cx(1, g.J, traj.shape[1] * traj.shape[2])
    loss = (AG.F(ops, traj, x) - y).abs().pow(2).sum()
    loss.backward()
    r = O.F_hat(g, x.detach().numpy()[0], traj.numpy()[0]).reshape(g.J, -1) - y.numpy()[0]
    ref = 2 * O.DFH_hat(g, x.detach().numpy()[0], r, traj.numpy()[0])
    assert np.allclose(x.grad.numpy()[0], ref, rtol=1e-10, atol=1e-10)
