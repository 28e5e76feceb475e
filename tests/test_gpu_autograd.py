"""Differentiation through the HIP operators (paper_1701_08361_amd.autograd):
gradients of least-squares losses through F_hat, DF and DF^H on the GPU
against the FP64 oracle's closed forms, and against central finite
differences of the GPU forward pass."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()            # fails loudly when the HIP library is missing
    return _t


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(torch, N=32, J=4, K=7, seed=31):
    from paper_1701_08361_amd import nlinv
    print(f"[case] autograd N={N} J={J} K={K} seed={seed}", flush=True)
    plan = nlinv.Plan(N, J, K)
    g = O.Geometry.make(N, J)
    traj = synth.radial_trajectory(N, K, 2 * N, 0, 1)
    x = synth.random_xhat(seed, g.R, J, g.Gc, 1.0, 0.3)
    dx = synth.random_xhat(seed + 1, g.R, J, g.Gc, 1.0, 0.3)
    y = synth.random_samples(seed + 2, J, K * 2 * N)
    tt = torch.from_numpy(traj[None].copy()).cuda()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a[None])).cuda()
    return plan, g, traj, tt, x, dx, y, dev


def test_grad_F_matches_oracle(torch):
    from paper_1701_08361_amd import autograd as AG
    plan, g, traj, tt, x, dx, y, dev = _case(torch)
    xt = dev(x).requires_grad_(True)
    loss = (AG.F(plan, tt, xt) - dev(y)).abs().pow(2).sum()
    loss.backward()
    r = O.F_hat(g, x.astype(np.complex128), traj).reshape(g.J, -1) - y
    ref = 2 * O.DFH_hat(g, x.astype(np.complex128), r, traj)
    e = rel(xt.grad.cpu().numpy()[0], ref)
    print(f"grad F rel {e:.2e}")
    assert e < GRAD_TOL


def test_grad_DF_matches_oracle(torch):
    from paper_1701_08361_amd import autograd as AG
    plan, g, traj, tt, x, dx, y, dev = _case(torch, seed=41)
    xt, dt = dev(x).requires_grad_(True), dev(dx).requires_grad_(True)
    loss = (AG.DF(plan, tt, xt, dt) - dev(y)).abs().pow(2).sum()
    loss.backward()
    xd, dd = x.astype(np.complex128), dx.astype(np.complex128)
    r = O.DF_hat(g, xd, dd, traj).reshape(g.J, -1) - y
    ex = rel(xt.grad.cpu().numpy()[0], 2 * O.DFH_hat(g, dd, r, traj))
    ed = rel(dt.grad.cpu().numpy()[0], 2 * O.DFH_hat(g, xd, r, traj))
    print(f"grad DF: x rel {ex:.2e}, dx rel {ed:.2e}")
    assert ex < GRAD_TOL and ed < GRAD_TOL


def test_grad_DFH_matches_oracle(torch):
    from paper_1701_08361_amd import autograd as AG
    plan, g, traj, tt, x, dx, y, dev = _case(torch, seed=51)
    xt, vt = dev(x).requires_grad_(True), dev(y).requires_grad_(True)
    w = dx
    loss = (AG.DFH(plan, tt, xt, vt) - dev(w)).abs().pow(2).sum()
    loss.backward()
    xd = x.astype(np.complex128)
    r = O.DFH_hat(g, xd, y, traj) - w
    ex = rel(xt.grad.cpu().numpy()[0], 2 * O.DFH_hat(g, r, y, traj))
    ev = rel(vt.grad.cpu().numpy()[0], 2 * O.DF_hat(g, xd, r, traj).reshape(g.J, -1))
    print(f"grad DFH: x rel {ex:.2e}, dy rel {ev:.2e}")
    assert ex < GRAD_TOL and ev < GRAD_TOL


def test_grad_F_finite_differences(torch):
    """Central differences of the float32 GPU loss agree with Re<grad, u>, for
    the gradient direction and two random directions.  The data are half the
    model output plus noise, so the loss is small against its slope and the
    float32 rounding of the loss stays far below the slope x step."""
    from paper_1701_08361_amd import autograd as AG
    plan, g, traj, tt, x, dx, y, dev = _case(torch, seed=61)
    ydata = (0.5 * O.F_hat(g, x.astype(np.complex128), traj).reshape(g.J, -1) + 0.01 * y).astype(np.complex64)
    xt = dev(x).requires_grad_(True)
    yt = dev(ydata)
    loss_of = lambda v: float((AG.F(plan, tt, v) - yt).abs().pow(2).sum())
    loss = (AG.F(plan, tt, xt) - yt).abs().pow(2).sum()
    loss.backward()
    grad = xt.grad.detach()
    scale = float(grad.abs().pow(2).sum().sqrt()) * float(np.linalg.norm(x))
    rng = np.random.default_rng(7)
    dirs = [grad / grad.abs().pow(2).sum().sqrt() * float(np.linalg.norm(x))]
    for k in range(2):
        u = rng.standard_normal(g.X) + 1j * rng.standard_normal(g.X)
        dirs.append(torch.from_numpy((u / np.linalg.norm(u) * np.linalg.norm(x)).astype(np.complex64)[None]).cuda())
    eps = 1e-3
    for k, u in enumerate(dirs):
        with torch.no_grad():
            fd = (loss_of(xt + eps * u) - loss_of(xt - eps * u)) / (2 * eps)
        an = float((grad.conj() * u).real.sum())
        print(f"direction {k}: finite difference {fd:.6e}, gradient {an:.6e}")
        assert abs(fd - an) <= 1e-3 * scale


def test_coil_synthesis_adjoint(torch):
    """nlinv_apply_WH against the oracle's W^-H, and <W^-1 c_hat, v> = <c_hat, W^-H v>."""
    from paper_1701_08361_amd import nlinv
    N, J = 64, 5
    print(f"[case] W^-H N={N} J={J}", flush=True)
    plan = nlinv.Plan(N, J, 5)
    g = O.Geometry.make(N, J)
    rng = np.random.default_rng(71)
    v = (rng.standard_normal((J, N, N)) + 1j * rng.standard_normal((J, N, N))).astype(np.complex64)
    out = plan.apply_WH(torch.from_numpy(v[None]).cuda()).cpu().numpy()[0]
    ref = g.pack(np.zeros((g.R, g.R)), O.winvh(v.astype(np.complex128), g.G, g.Gc, g.w))
    e = rel(out, ref)
    x = synth.random_xhat(72, g.R, J, g.Gc, 1.0, 1.0)
    c, _ = plan.coils(torch.from_numpy(x[None]).cuda(), want_img=False)
    lhs = np.vdot(c.cpu().numpy()[0].astype(np.complex128), v)
    rhs = np.vdot(x[g.R * g.R:].astype(np.complex128), out[g.R * g.R:].astype(np.complex128))
    print(f"W^-H rel {e:.2e}, adjoint mismatch {abs(lhs - rhs) / abs(lhs):.2e}")
    assert e < GRAD_TOL and abs(lhs - rhs) <= 1e-5 * abs(lhs)
    assert np.all(out[:g.R * g.R] == 0)


def _unrolled_case(torch, N=32, J=4, K=7, M=3, C=4):
    from paper_1701_08361_amd import nlinv
    s = synth.real_time_series(seed=73, N=N, J=J, J_phys=6, K=K, U=1, frames=1)
    plan = nlinv.Plan(N, J, K, U=1)
    g = O.Geometry.make(N, J)
    return plan, g, s


def test_unrolled_forward_matches_oracle(torch):
    """The unrolled form on the GPU (float32 operators, float32 CG algebra)
    against the oracle's IRGNM with the same counts."""
    from paper_1701_08361_amd import unrolled as UR
    N, J, K, M, C = 32, 4, 7, 3, 4
    print(f"[case] unrolled forward N={N} J={J} K={K} M={M} C={C}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K, M, C)
    traj = torch.from_numpy(s.traj).cuda()
    y = torch.from_numpy(s.y).cuda()
    with torch.no_grad():
        x = UR.reconstruct(plan, traj, y, g.R, newton=M, cg_iters=C)
        img = UR.image(plan, x, g.R)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(s.y[0], s.traj[0], g.R), P, newton=M, cg_iters=C)
    e = rel(img.cpu().numpy()[0], O.image(g, xr))
    print(f"unrolled image rel {e:.2e}")
    assert e < 1e-3


def test_unrolled_gradients_match_fp64(torch):
    """Gradients of ||image - phantom||^2 with respect to the data and alpha_0
    through 3 checkpointed Newton steps of 4 CG iterations: GPU (float32)
    against the same unrolled procedure in float64 on the oracle."""
    from paper_1701_08361_amd import unrolled as UR
    from test_autograd_cpu import OracleOps
    N, J, K, M, C = 32, 4, 7, 3, 4
    print(f"[case] unrolled gradients N={N} J={J} K={K} M={M} C={C}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K, M, C)
    truth = s.truth[0] * np.linalg.norm(s.coils.reshape(J, -1), axis=0).reshape(N, N)

    def grads(ops, traj, y0, dev, cdt, rdt):
        y = torch.from_numpy(y0).to(dev, cdt).requires_grad_(True)
        a0 = torch.tensor(1.0, dtype=rdt, device=dev, requires_grad=True)
        x = UR.reconstruct(ops, traj, y, g.R, newton=M, cg_iters=C, alpha0=a0)
        img = UR.image(ops, x, g.R)
        t = torch.from_numpy(truth).to(dev, rdt)
        loss = ((img[0] - t / t.norm() * img[0].detach().norm()) ** 2).sum()
        loss.backward()
        return y.grad.cpu().numpy(), float(a0.grad), float(loss.detach())

    gy, ga, L = grads(plan, torch.from_numpy(s.traj).cuda(), s.y, "cuda", torch.complex64, torch.float32)
    ry, ra, Lr = grads(OracleOps(g), torch.from_numpy(s.traj.astype(np.float64)), s.y.astype(np.complex128),
                       "cpu", torch.complex128, torch.float64)
    ey, ea = rel(gy, ry), abs(ga - ra) / abs(ra)
    print(f"loss {L:.6e} vs {Lr:.6e}; grad y rel {ey:.2e}; grad alpha0 {ga:.6e} vs {ra:.6e} (rel {ea:.2e})")
    assert ey < 1e-2 and ea < 1e-2


def test_unrolled_sobolev_weight_gradients_match_fp64(torch):
    """Another Sobolev weight w = (1 + a|k|^2)^l (a = 20, l = 2) built from the
    plan's (880, 16) operators: the forward image against the oracle's IRGNM
    defined with that weight, and the gradients of ||image - phantom||^2 with
    respect to a and l through 3 checkpointed Newton steps of 4 CG iterations,
    GPU (float32 operators) against the same procedure in float64 on the
    oracle."""
    from paper_1701_08361_amd import autograd as AG
    from paper_1701_08361_amd import unrolled as UR
    from test_autograd_cpu import OracleOps
    N, J, K, M, C = 32, 4, 7, 3, 4
    A, L = 20.0, 2.0
    print(f"[case] unrolled Sobolev-weight gradients N={N} J={J} K={K} M={M} C={C} a={A} l={L}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K, M, C)
    truth = s.truth[0] * np.linalg.norm(s.coils.reshape(J, -1), axis=0).reshape(N, N)

    def run(ops, traj, y0, dev, cdt, rdt):
        a = torch.tensor(A, dtype=torch.float64, device=dev, requires_grad=True)
        l = torch.tensor(L, dtype=torch.float64, device=dev, requires_grad=True)
        m = AG.Reweighted(ops, g.G, g.Gc, g.R, g.J, a, l)
        y = torch.from_numpy(y0).to(dev, cdt)
        x = UR.reconstruct(m, traj, y, g.R, newton=M, cg_iters=C)
        img = UR.image(m, x, g.R)
        t = torch.from_numpy(truth).to(dev, rdt)
        loss = ((img[0] - t / t.norm() * img[0].detach().norm()) ** 2).sum()
        loss.backward()
        return float(a.grad), float(l.grad), img.detach().cpu().numpy()[0]

    ga, gl, img = run(plan, torch.from_numpy(s.traj).cuda(), s.y, "cuda", torch.complex64, torch.float32)
    ra, rl, _ = run(OracleOps(g), torch.from_numpy(s.traj.astype(np.float64)), s.y.astype(np.complex128),
                    "cpu", torch.complex128, torch.float64)
    g2 = O.Geometry.make(N, J, a=A, l=L)
    P = O.psf_kernel(s.traj[0], g2.R, g2.G)
    xr = O.reconstruct(g2, O.grid(s.y[0], s.traj[0], g2.R), P, newton=M, cg_iters=C)
    e_img = rel(img, O.image(g2, xr))
    ea, el = abs(ga - ra) / abs(ra), abs(gl - rl) / abs(rl)
    print(f"image rel {e_img:.2e}; d/da {ga:.6e} vs {ra:.6e} (rel {ea:.2e}); d/dl {gl:.6e} vs {rl:.6e} (rel {el:.2e})")
    assert e_img < 1e-3
    assert ea < 1e-2 and el < 1e-2
