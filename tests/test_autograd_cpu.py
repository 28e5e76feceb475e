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
    """apply_F / apply_DF / apply_DFH, coils and apply_WH in the shapes of the
    C-ABI binding, FP64."""

    def __init__(self, g):
        self.g = g
        self.X = g.X

    def coils(self, xhat, want_img=False):
        return self._each(lambda x: self.g.coils(x), xhat), None

    def apply_WH(self, c):
        g = self.g
        def one(cj):
            return g.pack(np.zeros((g.R, g.R)), O.winvh(cj, g.G, g.Gc, g.w))
        return self._each(one, c)

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


def test_coils_gradcheck():
    ops, traj, g, cx = _setup(seed=4)
    x = cx(2, g.X).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: AG.coils(ops, x), (x,), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_unrolled_equals_oracle_reconstruction():
    """The unrolled form (operators F and F^H separately) reproduces the
    oracle's IRGNM (normal operator through the PSF convolution): the same
    iteration, since T = F^H F exactly."""
    from paper_1701_08361_amd import unrolled as UR
    ops, traj, g, cx = _setup(B=1, N=8, J=2, K=5, seed=5)
    s = synth.single_frame(seed=5, N=8, J=2, K=5)
    t = s.traj.astype(np.float64)
    y = torch.from_numpy(s.y.astype(np.complex128))
    x = UR.reconstruct(ops, torch.from_numpy(t), y, g.R, newton=3, cg_iters=4, checkpoint_steps=True)
    P = O.psf_kernel(t[0], g.R, g.G)
    ref = O.reconstruct(g, O.grid(s.y[0].astype(np.complex128), t[0], g.R), P, newton=3, cg_iters=4)
    err = np.linalg.norm(x.numpy()[0] - ref) / np.linalg.norm(ref)
    assert err < 1e-9, err


def test_unrolled_gradcheck_data_and_alpha():
    """Finite-difference check of d image / d (y, alpha_0) through 2 Newton steps
    of 2 CG iterations, each step checkpointed."""
    from paper_1701_08361_amd import unrolled as UR
    ops, traj, g, cx = _setup(B=1, N=8, J=2, K=3, seed=6)
    y = (0.3 * cx(1, g.J, traj.shape[1] * traj.shape[2])).requires_grad_(True)
    a0 = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)

    def fn(y, a0):
        x = UR.reconstruct(ops, traj[:1], y, g.R, newton=2, cg_iters=2, alpha0=a0)
        return UR.image(ops, x, g.R)

    assert torch.autograd.gradcheck(fn, (y, a0), eps=1e-6, atol=1e-5, rtol=1e-4)


# --------------------------------------------------------------------------
# another Sobolev weight (Sec. 3.2, Fig. weight_func), differentiable in a, l
# --------------------------------------------------------------------------

A_W, L_W = 20.0, 2.0       # a soft weight under test; the operators are built for (880, 16)


def _reweighted(ops, g, a=A_W, l=L_W):
    a = torch.as_tensor(a, dtype=torch.float64)
    l = torch.as_tensor(l, dtype=torch.float64)
    return AG.Reweighted(ops, g.G, g.Gc, g.R, g.J, a, l)


def test_reweighted_operators_equal_the_oracle_at_that_weight():
    """F, DF, DF^H and the coil synthesis rebuilt from the (880, 16) operators
    equal the oracle's operators defined with w = (1 + 20|k|^2)^2."""
    ops, traj, g, cx = _setup(B=2, N=8, J=2, K=3, seed=11)
    g2 = O.Geometry.make(8, 2, a=A_W, l=L_W)
    ops2 = OracleOps(g2)
    m = _reweighted(ops, g)
    rng = np.random.default_rng(11)
    x = torch.from_numpy(np.stack([g2.pack(rng.standard_normal((g2.R, g2.R)) + 0j,
                                           (rng.standard_normal((g2.J, g2.Gc, g2.Gc)) + 1j) * g2.w[None])
                                   for _ in range(2)]))
    dx = torch.from_numpy(np.stack([g2.pack(rng.standard_normal((g2.R, g2.R)) + 1j,
                                            rng.standard_normal((g2.J, g2.Gc, g2.Gc)) * g2.w[None] + 0j)
                                    for _ in range(2)]))
    S = traj.shape[1] * traj.shape[2]
    dy = cx(2, g.J, S)
    rel = lambda u, v: float(torch.linalg.norm(u - v) / torch.linalg.norm(v))
    assert rel(m.F(traj, x), ops2.apply_F(traj, x)) < 1e-12
    assert rel(m.DF(traj, x, dx), ops2.apply_DF(traj, x, dx)) < 1e-12
    assert rel(m.DFH(traj, x, dy), ops2.apply_DFH(traj, x, dy)) < 1e-12
    assert rel(m.coils(x), ops2.coils(x)[0]) < 1e-12
    # at the reference weight the rescaling is the identity
    m0 = _reweighted(ops, g, 880.0, 16.0)
    assert torch.equal(m0.d, torch.ones_like(m0.d))


def test_unrolled_reweighted_equals_oracle_reconstruction():
    """The unrolled IRGNM under (20, 2), from the (880, 16) operators,
    reproduces the oracle's IRGNM with that weight."""
    from paper_1701_08361_amd import unrolled as UR
    ops, traj, g, cx = _setup(B=1, N=8, J=2, K=5, seed=5)
    g2 = O.Geometry.make(8, 2, a=A_W, l=L_W)
    s = synth.single_frame(seed=5, N=8, J=2, K=5)
    t = s.traj.astype(np.float64)
    y = torch.from_numpy(s.y.astype(np.complex128))
    x = UR.reconstruct(_reweighted(ops, g), torch.from_numpy(t), y, g.R, newton=3, cg_iters=4)
    P = O.psf_kernel(t[0], g2.R, g2.G)
    ref = O.reconstruct(g2, O.grid(s.y[0].astype(np.complex128), t[0], g2.R), P, newton=3, cg_iters=4)
    err = np.linalg.norm(x.detach().numpy()[0] - ref) / np.linalg.norm(ref)
    assert err < 1e-9, err
    # and the weight matters: the (880, 16) reconstruction differs
    ref0 = O.reconstruct(g, O.grid(s.y[0].astype(np.complex128), t[0], g.R), P, newton=3, cg_iters=4)
    assert np.linalg.norm(ref0 - ref) > 1e-3 * np.linalg.norm(ref)


def test_unrolled_gradcheck_sobolev_weight():
    """Finite-difference check of d image / d (a, l) of the Sobolev weight
    through 2 Newton steps of 2 CG iterations, each step checkpointed."""
    from paper_1701_08361_amd import unrolled as UR
    ops, traj, g, cx = _setup(B=1, N=8, J=2, K=3, seed=7)
    y = 0.3 * cx(1, g.J, traj.shape[1] * traj.shape[2])
    a = torch.tensor(A_W, dtype=torch.float64, requires_grad=True)
    l = torch.tensor(L_W, dtype=torch.float64, requires_grad=True)

    def fn(a, l):
        m = AG.Reweighted(ops, g.G, g.Gc, g.R, g.J, a, l)
        x = UR.reconstruct(m, traj[:1], y, g.R, newton=2, cg_iters=2)
        return UR.image(m, x, g.R)

    # the weight reaches the image: a gradient far from zero is checked
    ga, gl = torch.autograd.grad(fn(a, l).sum(), (a, l))
    print(f"d sum(image) / d(a, l) = {float(ga):.3e}, {float(gl):.3e}")
    assert abs(float(ga)) > 1e-4 and abs(float(gl)) > 1e-3
    assert torch.autograd.gradcheck(fn, (a, l), eps=1e-5, atol=1e-6, rtol=1e-4)
