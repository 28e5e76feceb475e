"""Differentiation through the HIP operators (paper_1701_08361_amd.autograd):
gradients of least-squares losses through F_hat, DF and DF^H on the GPU
against the FP64 oracle's closed forms, and against central finite
differences of the GPU forward pass; the operators of the Toeplitz form
(gridding, E_x, E_x^H, E_x^H T E_x) against the oracle; and the unrolled
IRGNM in the Toeplitz form, forward and gradients, against the same
procedure in FP64 on the oracle (32 px) and against the oracle's FP64
finite differences stored for a 160 px, 5 Newton x 20 CG case."""
import json
import os

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


def _toeplitz_plan(torch, N=32, J=4, K=7, B=2, seed=81):
    """A plan of batch B with the PSF kernel of item b's trajectory at turn b."""
    from paper_1701_08361_amd import nlinv
    plan = nlinv.Plan(N, J, K, U=B, batch=B)
    g = O.Geometry.make(N, J)
    traj = np.stack([synth.radial_trajectory(N, K, 2 * N, b, B) for b in range(B)])
    tt = torch.from_numpy(traj).cuda()
    for b in range(B):
        plan.psf(tt[b], b)
    return plan, g, traj, tt


def test_toeplitz_form_operators_match_oracle(torch):
    """z = F^H y, F img, E_x p, E_x^H img and E_xa^H T E_xb p + alpha p (batch 2,
    two turns, xa != xb) against the oracle's operators, <= 1e-4."""
    from test_autograd_cpu import OracleOps
    N, J, K, B = 32, 4, 7, 2
    print(f"[case] Toeplitz-form operators N={N} J={J} K={K} B={B}", flush=True)
    plan, g, traj, tt = _toeplitz_plan(torch, N, J, K, B)
    ref = OracleOps(g, traj.astype(np.float64))
    t64 = torch.from_numpy(traj.astype(np.float64))
    rng = np.random.default_rng(82)
    xa = np.stack([synth.random_xhat(83 + b, g.R, J, g.Gc, 1.0, 0.3) for b in range(B)])
    xb = np.stack([synth.random_xhat(85 + b, g.R, J, g.Gc, 1.0, 0.3) for b in range(B)])
    p = np.stack([synth.random_xhat(87 + b, g.R, J, g.Gc, 1.0, 0.3) for b in range(B)]).astype(np.complex128)
    y = np.stack([synth.random_samples(89 + b, J, K * 2 * N) for b in range(B)])
    img = (rng.standard_normal((B, J, N, N)) + 1j * rng.standard_normal((B, J, N, N))).astype(np.complex64)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c128 = lambda a: torch.from_numpy(np.asarray(a, np.complex128))
    errs = {
        "grid": rel(plan.grid(tt, cu(y)).cpu().numpy(), ref.grid(t64, c128(y)).numpy()),
        "nudft": rel(plan.nudft(tt, cu(img)).cpu().numpy(), ref.nudft(t64, c128(img)).numpy()),
        "E": rel(plan.apply_E(cu(xa), cu(p)).cpu().numpy(), ref.apply_E(c128(xa), c128(p)).numpy()),
        "EH": rel(plan.apply_EH(cu(xa), cu(img)).cpu().numpy(), ref.apply_EH(c128(xa), c128(img)).numpy()),
        "normal2": rel(plan.apply_normal2([0, 1], cu(xa), cu(xb), cu(p), 0.3).cpu().numpy(),
                       ref.apply_normal2([0, 1], c128(xa), c128(xb), c128(p), 0.3).numpy()),
        "normal2 swapped turns": rel(plan.apply_normal2([1, 0], cu(xa), cu(xb), cu(p), 0.0).cpu().numpy(),
                                     ref.apply_normal2([1, 0], c128(xa), c128(xb), c128(p), 0.0).numpy()),
    }
    print("; ".join(f"{k} rel {v:.2e}" for k, v in errs.items()))
    assert all(v < 1e-4 for v in errs.values())
    # with xa = xb the operator equals nlinv_apply_normal up to p's storage precision
    q1 = plan.apply_normal2([0, 1], cu(xa), cu(xa), cu(p.astype(np.complex64).astype(np.complex128)), 0.3)
    q0 = plan.apply_normal([0, 1], cu(xa), cu(p.astype(np.complex64)), 0.3)
    e = rel(q1.cpu().numpy(), q0.cpu().numpy().astype(np.complex128))
    print(f"normal2(x, x) vs apply_normal rel {e:.2e}")
    assert e < 1e-5
    plan.close()


def test_newton_step_equals_the_solvers_steps(torch):
    """nlinv_newton_step with alpha_n and the plan's CG count, M times from the
    unit start, equals nlinv_reconstruct bit for bit (both forms of the CG
    iteration); and a plan of weight (20, 2) equals the (880, 16) plan under
    the coil-weight table of (20, 2) up to the table's float32 rounding, and
    the plan's own table restores its own bits."""
    from paper_1701_08361_amd import autograd as AG
    from paper_1701_08361_amd import nlinv
    N, J, K, M, C = 32, 4, 7, 3, 5
    print(f"[case] Newton step N={N} J={J} K={K} M={M} C={C}", flush=True)
    s = synth.real_time_series(seed=75, N=N, J=J, J_phys=6, K=K, U=1, frames=1)
    tr, y = torch.from_numpy(s.traj).cuda(), torch.from_numpy(s.y).cuda()
    for passes in (6, 4):
        plan = nlinv.Plan(N, J, K, newton=M, cg=C, cg_passes=passes)
        z = plan.grid(tr, y, turns=[0])
        ref, _, _ = plan.reconstruct(z, [0])
        x = torch.zeros(1, plan.X, dtype=torch.complex64, device="cuda")
        x[:, :plan.R * plan.R] = 1
        for n in range(M):
            plan.newton_step([0], z, x, 0.5 ** n, C)
        assert torch.equal(x, ref), passes
        plan.close()
    g = O.Geometry.make(N, J)
    p20 = nlinv.Plan(N, J, K, newton=M, cg=C, sob_a=20.0, sob_l=2.0)
    z = p20.grid(tr, y, turns=[0])
    x20, _, _ = p20.reconstruct(z, [0])
    plan = nlinv.Plan(N, J, K, newton=M, cg=C)
    plan.psf(tr[0], 0)
    own, _, _ = plan.reconstruct(z, [0])
    m = AG.Reweighted(plan, g.G, g.Gc, g.R, J, torch.tensor(20.0, dtype=torch.float64, device="cuda"),
                      torch.tensor(2.0, dtype=torch.float64, device="cuda"))
    plan.set_coil_weights(m.winv)
    xw, _, _ = plan.reconstruct(z, [0])
    plan.set_coil_weights(None)
    back, _, _ = plan.reconstruct(z, [0])
    e = rel(xw.cpu().numpy(), x20.cpu().numpy())
    print(f"coil-weight table (20, 2) vs plan of (20, 2): rel {e:.2e}")
    assert e < 1e-5 and torch.equal(back, own)
    # with HIP graphs: a captured reconstruction is not replayed with a stale table
    plan.set_graphs(True)
    g_own, _, _ = plan.reconstruct(z, [0])
    plan.set_coil_weights(m.winv)
    g_w, _, _ = plan.reconstruct(z, [0])
    plan.set_coil_weights(None)
    g_back, _, _ = plan.reconstruct(z, [0])
    torch.cuda.synchronize()
    assert torch.equal(g_own, own) and torch.equal(g_w, xw) and torch.equal(g_back, own)
    assert rel(own.cpu().numpy(), x20.cpu().numpy()) > 1e-3     # the weight matters
    p20.close()
    plan.close()


def _unrolled_case(torch, N=32, J=4, K=7, seed=73):
    from paper_1701_08361_amd import nlinv
    s = synth.real_time_series(seed=seed, N=N, J=J, J_phys=6 if N < 64 else 30, K=K, U=1, frames=1)
    plan = nlinv.Plan(N, J, K, U=1)
    plan.psf(torch.from_numpy(s.traj[0]).cuda(), 0)
    g = O.Geometry.make(N, J)
    return plan, g, s


def test_unrolled_forward_matches_oracle(torch):
    """The unrolled Toeplitz form on the GPU (library operators, FP64 CG
    algebra) against the oracle's IRGNM with the same counts; the nudft form
    (F and F^H separately) too."""
    from paper_1701_08361_amd import unrolled as UR
    N, J, K, M, C = 32, 4, 7, 3, 4
    print(f"[case] unrolled forward N={N} J={J} K={K} M={M} C={C}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K)
    traj = torch.from_numpy(s.traj).cuda()
    y = torch.from_numpy(s.y).cuda()
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(s.y[0], s.traj[0], g.R), P, newton=M, cg_iters=C)
    with torch.no_grad():
        e = {}
        for form in ("toeplitz", "nudft"):
            x = UR.reconstruct(plan, traj, y, g.R, newton=M, cg_iters=C, form=form, turns=[0])
            e[form] = rel(UR.image(plan, x, g.R).cpu().numpy()[0], O.image(g, xr))
    print(f"unrolled image rel: Toeplitz form {e['toeplitz']:.2e}, nudft form {e['nudft']:.2e}")
    assert e["toeplitz"] < 1e-4 and e["nudft"] < 1e-3
    plan.close()


TRUTH_LOSS = "||image - phantom||^2"


def _loss(torch, img, truth):
    t = torch.from_numpy(truth).to(img.device, img.dtype)
    return ((img[0] - t) ** 2).sum()


def test_unrolled_gradients_match_fp64(torch):
    """Gradients of ||image - phantom||^2 with respect to the data y, alpha_0
    and the Sobolev weight's a and l (w = (1 + a|k|^2)^l, here a = 20, l = 2,
    rebuilt from the plan's (880, 16) operators) through 3 checkpointed Newton
    steps of 4 CG iterations in the Toeplitz form: GPU against the same
    procedure in FP64 with the oracle's operators, <= 1e-3."""
    from paper_1701_08361_amd import autograd as AG
    from paper_1701_08361_amd import unrolled as UR
    from test_autograd_cpu import OracleOps
    N, J, K, M, C = 32, 4, 7, 3, 4
    A, L = 20.0, 2.0
    print(f"[case] unrolled gradients N={N} J={J} K={K} M={M} C={C} a={A} l={L}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K)
    truth = s.truth[0] * np.linalg.norm(s.coils.reshape(J, -1), axis=0).reshape(N, N)

    def run(ops, traj, y0, dev, cdt):
        y = torch.from_numpy(y0).to(dev, cdt).requires_grad_(True)
        a0 = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
        a = torch.tensor(A, dtype=torch.float64, device=dev, requires_grad=True)
        l = torch.tensor(L, dtype=torch.float64, device=dev, requires_grad=True)
        m = AG.Reweighted(ops, g.G, g.Gc, g.R, g.J, a, l)
        x = UR.reconstruct(m, traj, y, g.R, newton=M, cg_iters=C, alpha0=a0, turns=[0])
        img = UR.image(m, x, g.R)
        loss = _loss(torch, img, truth)
        loss.backward()
        return (y.grad.cpu().numpy().astype(np.complex128), float(a0.grad), float(a.grad), float(l.grad),
                float(loss.detach()), img.detach().cpu().numpy()[0])

    gy, ga0, ga, gl, Lg, img = run(plan, torch.from_numpy(s.traj).cuda(), s.y, "cuda", torch.complex64)
    ry, ra0, ra, rl, Lr, _ = run(OracleOps(g, s.traj.astype(np.float64)), torch.from_numpy(s.traj.astype(np.float64)),
                                 s.y.astype(np.complex128), "cpu", torch.complex128)
    g2 = O.Geometry.make(N, J, a=A, l=L)
    xr = O.reconstruct(g2, O.grid(s.y[0], s.traj[0], g2.R), O.psf_kernel(s.traj[0], g2.R, g2.G), newton=M,
                       cg_iters=C)
    e_img = rel(img, O.image(g2, xr))
    e = {"y": rel(gy, ry), "alpha0": abs(ga0 - ra0) / abs(ra0), "a": abs(ga - ra) / abs(ra),
         "l": abs(gl - rl) / abs(rl)}
    print(f"loss {Lg:.6e} vs {Lr:.6e}; image rel {e_img:.2e}; "
          + "; ".join(f"grad {k} rel {v:.2e}" for k, v in e.items())
          + f"; d/d alpha0 {ga0:.6e} vs {ra0:.6e}; d/da {ga:.6e} vs {ra:.6e}; d/dl {gl:.6e} vs {rl:.6e}")
    assert e_img < 1e-4
    assert all(v < 1e-3 for v in e.values())
    plan.close()


GOLDEN_160 = os.path.join(os.path.dirname(__file__), "golden", "unrolled160.json")


def test_unrolled_160px_five_newton_against_oracle_differences(torch):
    """160 px, 10 coils, 15 spokes, 5 Newton x 20 CG in the Toeplitz form,
    loss ||image - phantom||^2: the loss, sampled image pixels, the
    derivatives in alpha_0, a and l, and the data gradient's projections on
    eight seeded directions against the oracle's FP64 reconstruction and its
    central differences (tests/golden/unrolled160.json, written by
    make_unrolled160.py).  The data gradient is measured by
    sqrt(sum_k (g.u_k - d_k)^2 / sum_k d_k^2): for random directions both
    sums estimate ||g - grad||^2 and ||grad||^2 up to the same factor, so the
    ratio estimates the gradient's relative error; a single projection can
    be small and make its own relative error large."""
    from paper_1701_08361_amd import autograd as AG
    from paper_1701_08361_amd import unrolled as UR
    with open(GOLDEN_160) as f:
        gold = json.load(f)
    c = gold["case"]
    N, J, K, M, C = c["N"], c["J"], c["K"], c["newton"], c["cg"]
    print(f"[case] unrolled 160 px N={N} J={J} K={K} M={M} C={C}", flush=True)
    plan, g, s = _unrolled_case(torch, N, J, K, seed=c["seed"])
    truth = s.truth[0] * np.linalg.norm(s.coils.reshape(J, -1), axis=0).reshape(N, N) * c["truth_scale"]
    y = torch.from_numpy(s.y).cuda().requires_grad_(True)
    a0 = torch.tensor(c["alpha0"], dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(c["a"], dtype=torch.float64, device="cuda", requires_grad=True)
    l = torch.tensor(c["l"], dtype=torch.float64, device="cuda", requires_grad=True)
    m = AG.Reweighted(plan, g.G, g.Gc, g.R, g.J, a, l)
    x = UR.reconstruct(m, torch.from_numpy(s.traj).cuda(), y, g.R, newton=M, cg_iters=C, alpha0=a0, turns=[0])
    img = UR.image(m, x, g.R)
    loss = _loss(torch, img, truth)
    loss.backward()
    im = img.detach().cpu().numpy()[0].ravel()
    idx = np.asarray(gold["pixels"]["index"])
    e_pix = float(np.max(np.abs(im[idx] - np.asarray(gold["pixels"]["value"])))) / gold["image_norm"]
    e_norm = abs(float(np.linalg.norm(im)) - gold["image_norm"]) / gold["image_norm"]
    e_loss = abs(float(loss) - gold["loss"]) / gold["loss"]
    ref = gold["derivatives"]
    got = {"alpha0": float(a0.grad), "a": float(a.grad), "l": float(l.grad)}
    e = {k: abs(got[k] - ref[k]) / abs(ref[k]) for k in got}
    gy = y.grad.cpu().numpy().astype(np.complex128)
    num = den = 0.0
    for k, d in enumerate(gold["data_directions"]):
        u = synth.random_samples(d["seed"], J, s.y.shape[-1]).astype(np.complex128)
        gu = float(np.real(np.vdot(gy[0], u)))
        num += (gu - ref[f"y.u{k}"]) ** 2
        den += ref[f"y.u{k}"] ** 2
        print(f"  y.u{k}: {gu:.6e} vs {ref[f'y.u{k}']:.6e}")
    e["y"] = float(np.sqrt(num / den))
    print(f"loss {float(loss):.6e} vs {gold['loss']:.6e} (rel {e_loss:.2e}); image norm rel {e_norm:.2e}; "
          f"sampled pixels max rel {e_pix:.2e}; "
          + "; ".join(f"{k} {got[k]:.6e} vs {ref[k]:.6e}" for k in got)
          + "; relative errors " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e_norm < 1e-4 and e_pix < 1e-4 and e_loss < 1e-3
    assert all(v < TOL_160 for v in e.values())
    plan.close()


TOL_160 = 1e-3
