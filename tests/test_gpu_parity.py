"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: relative L2 error <= 1e-4 for every operator application and
<= 1e-3 on the final image |rho| sqrt(sum |c_j|^2) and on the gauge-invariant
coil images rho c_j after a fixed number of Newton steps.  Inputs are the
seeded synthetic series of the generator; nothing is read from stored GPU
output.
"""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

OP_TOL = 1e-4
IMG_TOL = 1e-3


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()            # fails loudly when the HIP library is missing
    return _t


def nl():
    from paper_1701_08361_amd import nlinv
    return nlinv


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_point(seed, g, c_scale=1.0):
    """x_hat with O(1) image and coil spectra (complex64)."""
    return synth.random_xhat(seed, g.R, g.J, g.Gc, 1.0, c_scale)


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


# ---------------------------------------------------------------------------
# gridding, coils, PSF convolution
# ---------------------------------------------------------------------------

def test_grid_ragged_readout(torch):
    """A readout length that is not 2N (odd, 77 samples per spoke): the
    Kaiser-Bessel tables and the exact sum against the oracle's sum."""
    N, J, K, S_r = 32, 3, 7, 77
    print_case("grid ragged", N=N, J=J, K=K, S_r=S_r)
    s = synth.single_frame(seed=13, N=N, J=J, K=K, S_r=S_r)
    assert s.traj.shape[2] == S_r
    ref = O.grid(s.y[0], s.traj[0], N)
    for flags in (0, 2):
        plan = nl().Plan(N, J, K, S_r=S_r, flags=flags)
        z = host(plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0]))
        print(f"grid ragged flags={flags}: rel {rel(z[0], ref):.2e}")
        assert rel(z[0], ref) < 1e-6


@pytest.mark.parametrize("N,J,K,seed", [(32, 3, 5, 11), (64, 8, 13, 1), (160, 10, 15, 2),
                                        (240, 3, 5, 4)])   # partial 32 x 32 pixel tiles
def test_grid_matches_exact_adjoint_nudft(torch, N, J, K, seed):
    """Kaiser-Bessel gridding (turns given, the default) and the exact sum
    (NLINV_F_EXACT_GRID, and calls without turns) against the oracle's exact sum."""
    print_case("grid", N=N, J=J, K=K, seed=seed)
    s = synth.single_frame(seed=seed, N=N, J=J, K=K)
    ref = O.grid(s.y[0], s.traj[0], N)
    for flags in (0, 2):
        plan = nl().Plan(N, J, K, flags=flags)
        z = host(plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0]))
        ze = host(plan.grid(dev(torch, s.traj), dev(torch, s.y)))
        print(f"grid flags={flags}: rel {rel(z[0], ref):.2e}, exact path {rel(ze[0], ref):.2e}")
        assert rel(z[0], ref) < OP_TOL and rel(ze[0], ref) < OP_TOL
        # the gridding error sits at float32 rounding, far inside the operator bar
        assert rel(z[0], ref) < 1e-6


def test_grid_tables_are_reproducible_and_handle_long_rows(torch):
    """The per-turn gridding tables are built on the device (count, scan,
    atomic fill, per-row sort by sample index): rebuilding a turn, building it
    in another plan, or after another trajectory gives the same gridded data
    bit for bit; and a trajectory whose 15 spokes coincide (rows of ~135
    entries, more than one wavefront's width) grids to the exact sum."""
    N, J, K = 64, 4, 15
    print_case("grid tables", N=N, J=J, K=K)
    s = synth.single_frame(seed=21, N=N, J=J, K=K)
    s2 = synth.single_frame(seed=22, N=N, J=J, K=K)
    tr, y = dev(torch, s.traj), dev(torch, s.y)
    plan = nl().Plan(N, J, K)
    z0 = host(plan.grid(tr, y, turns=[0]))
    plan.psf(tr[0], 0)
    z1 = host(plan.grid(tr, y, turns=[0]))
    plan.psf(dev(torch, s2.traj[0]), 0)
    plan.psf(tr[0], 0)
    z2 = host(plan.grid(tr, y, turns=[0]))
    other = nl().Plan(N, J, K, U=2)
    other.psf(dev(torch, s2.traj[0]), 0)
    z3 = host(other.grid(tr, y, turns=[1]))
    assert np.array_equal(z0, z1) and np.array_equal(z0, z2) and np.array_equal(z0, z3)
    # coinciding spokes
    same = np.repeat(s.traj[0][:1], K, axis=0)[None]
    ref = O.grid(s.y[0], same[0], N)
    plan2 = nl().Plan(N, J, K)
    z = host(plan2.grid(dev(torch, same), y, turns=[0]))
    zb = host(plan2.grid(dev(torch, same), y, turns=[0]))
    print(f"coinciding spokes: rel {rel(z[0], ref):.2e}")
    assert rel(z[0], ref) < 1e-6 and np.array_equal(z, zb)
    for p_ in (plan, other, plan2):
        p_.close()


@pytest.mark.parametrize("N,J", [(32, 2), (64, 8), (128, 5), (160, 10), (192, 3), (224, 4), (240, 3), (256, 2)])
def test_coil_synthesis(torch, N, J):
    print_case("coils", N=N, J=J)
    plan = nl().Plan(N, J, 5)
    g = O.Geometry.make(N, J)
    x = random_point(100 + N, g)
    co, img = plan.coils(dev(torch, x[None]))
    ref = g.coils(x)
    assert rel(host(co)[0], ref) < OP_TOL
    assert rel(host(img)[0], O.image(g, x)) < OP_TOL


def _normal_case(torch, N, J, K, U, B, alpha, seed):
    plan = nl().Plan(N, J, K, U=U, batch=B)
    g = O.Geometry.make(N, J)
    trajs = [synth.radial_trajectory(N, K, 2 * N, t, U) for t in range(U)]
    for t in range(U):
        plan.psf(dev(torch, trajs[t]), t)
    turns = [(b * 2 + 1) % U for b in range(B)]
    xs = np.stack([random_point(seed + b, g) for b in range(B)])
    ps = np.stack([random_point(seed + 50 + b, g) for b in range(B)])
    q = host(plan.apply_normal(turns, dev(torch, xs), dev(torch, ps), alpha=alpha))
    R2 = g.R * g.R
    for b in range(B):
        P = O.psf_kernel(trajs[turns[b]], g.R, g.G)
        ref = O.normal(g, xs[b], ps[b], P) + alpha * ps[b].astype(np.complex128)
        print(f"normal item {b}: image block rel {rel(q[b, :R2], ref[:R2]):.2e}  "
              f"coil block rel {rel(q[b, R2:], ref[R2:]):.2e}")
        assert rel(q[b, :R2], ref[:R2]) < OP_TOL, "image block"
        assert rel(q[b, R2:], ref[R2:]) < OP_TOL, "coil block"
        # scale-free check of every coil coefficient (undo the Sobolev weight)
        if alpha == 0.0:
            w = np.tile(g.w.ravel(), J)
            assert rel(q[b, R2:] * w, ref[R2:] * w) < OP_TOL, "weighted coil block"


@pytest.mark.parametrize("N,J,K,U,B,alpha", [
    (32, 2, 5, 1, 1, 0.0), (64, 8, 13, 2, 3, 0.37), (64, 8, 13, 1, 1, 0.0),
    (128, 4, 11, 3, 2, 0.0), (160, 10, 15, 5, 2, 0.125), (192, 3, 9, 1, 1, 0.0),
    (216, 4, 13, 2, 2, 0.3),    # 432 grid (16 x 27 team transform)
    (224, 5, 21, 2, 2, 0.5), (240, 3, 9, 1, 1, 0.25), (256, 2, 11, 2, 2, 0.0),
    (32, 64, 5, 2, 2, 0.1),     # the most channels a plan takes
    (32, 2, 3, 4, 64, 0.0)])    # the largest batch
def test_normal_operator(torch, N, J, K, U, B, alpha):
    print_case("normal", N=N, J=J, K=K, U=U, B=B, alpha=alpha)
    _normal_case(torch, N, J, K, U, B, alpha, seed=7 * N + J)


# ---------------------------------------------------------------------------
# operators on radial samples
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,J,K,B", [(32, 2, 5, 1), (64, 8, 13, 2), (160, 10, 15, 1),
                                     (240, 2, 5, 1)])   # field of view not a multiple of the x chunk
def test_F_DF_DFH_match_oracle(torch, N, J, K, B):
    print_case("F/DF/DFH", N=N, J=J, K=K, B=B)
    plan = nl().Plan(N, J, K, batch=B)
    g = O.Geometry.make(N, J)
    trajs = np.stack([synth.radial_trajectory(N, K, 2 * N, b, 3) for b in range(B)])
    xs = np.stack([random_point(300 + b, g) for b in range(B)])
    dxs = np.stack([random_point(400 + b, g) for b in range(B)])
    vs = np.stack([synth.random_samples(500 + b, J, plan.S) for b in range(B)])
    tr = dev(torch, trajs)
    Fx = host(plan.apply_F(tr, dev(torch, xs)))
    DFu = host(plan.apply_DF(tr, dev(torch, xs), dev(torch, dxs)))
    DFHv = host(plan.apply_DFH(tr, dev(torch, xs), dev(torch, vs)))
    R2 = g.R * g.R
    for b in range(B):
        assert rel(Fx[b], O.F_hat(g, xs[b], trajs[b])) < OP_TOL
        assert rel(DFu[b], O.DF_hat(g, xs[b], dxs[b], trajs[b])) < OP_TOL
        ref = O.DFH_hat(g, xs[b], vs[b], trajs[b])
        assert rel(DFHv[b, :R2], ref[:R2]) < OP_TOL
        assert rel(DFHv[b, R2:], ref[R2:]) < OP_TOL


def test_gpu_DF_DFH_are_adjoint(torch):
    N, J, K = 64, 4, 9
    plan = nl().Plan(N, J, K)
    g = O.Geometry.make(N, J)
    tr = dev(torch, synth.radial_trajectory(N, K, 2 * N, 0, 1)[None])
    x = dev(torch, random_point(1, g)[None])
    u = dev(torch, random_point(2, g)[None])
    v = dev(torch, synth.random_samples(3, J, plan.S)[None])
    lhs = torch.vdot(plan.apply_DF(tr, x, u).ravel().to(torch.complex128), v.ravel().to(torch.complex128))
    rhs = torch.vdot(u.ravel().to(torch.complex128), plan.apply_DFH(tr, x, v).ravel().to(torch.complex128))
    assert abs(complex(lhs) - complex(rhs)) < 1e-5 * abs(complex(lhs))


# ---------------------------------------------------------------------------
# reconstruction
# ---------------------------------------------------------------------------

def _recon_compare(g, x_gpu, img_gpu, x_ref):
    img_ref = O.image(g, x_ref)
    e_img = rel(img_gpu, img_ref)
    e_rc = rel(O.coil_images(g, x_gpu), O.coil_images(g, x_ref))
    return e_img, e_rc


def test_reconstruct_single_frame_c1(torch):
    """Plain single frame: 64 px, 128 grid, 8 coils, 13 spokes x 128, 7 x 10."""
    print_case("recon c1", N=64, J=8, K=13, M=7, C=10)
    s = synth.single_frame(seed=1)
    plan = nl().Plan(64, 8, 13, newton=7, cg=10)
    z = plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0])
    x, img, _ = plan.reconstruct(z, [0], want_img=True)
    g = O.Geometry.make(64, 8)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(s.y[0], s.traj[0], g.R), P, newton=7, cg_iters=10)
    e_img, e_rc = _recon_compare(g, host(x)[0], host(img)[0], xr)
    print(f"c1 image rel {e_img:.2e}  rho*c rel {e_rc:.2e}")
    assert e_img < IMG_TOL and e_rc < IMG_TOL


@pytest.mark.parametrize("N,J,K,M,C", [
    (128, 8, 11, 4, 8),     # smallest mixed-size configuration (256 grid)
    (192, 16, 21, 3, 6),    # largest mixed-size configuration (384 grid, 16 coils, 21 spokes)
    (216, 6, 13, 2, 4),     # 432 grid (16 x 27)
    (224, 16, 21, 2, 4),    # 448 grid, 16 coils
    (256, 4, 9, 2, 3),      # largest supported grid (512)
    (32, 1, 1, 3, 4),       # degenerate: one coil, one spoke
    (32, 64, 5, 2, 3),      # the most channels a plan takes
])
def test_reconstruct_sizes(torch, N, J, K, M, C):
    """Single frames across the supported grid sizes and the degenerate case,
    Kaiser-Bessel gridding included, against the oracle."""
    print_case("recon sizes", N=N, J=J, K=K, M=M, C=C)
    s = synth.single_frame(seed=3, N=N, J=J, K=K)
    plan = nl().Plan(N, J, K, newton=M, cg=C)
    z = plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0])
    x, img, _ = plan.reconstruct(z, [0], want_img=True)
    g = O.Geometry.make(N, J)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(s.y[0], s.traj[0], g.R), P, newton=M, cg_iters=C)
    e_img, e_rc = _recon_compare(g, host(x)[0], host(img)[0], xr)
    print(f"sizes N={N} J={J} K={K}: image rel {e_img:.2e}  rho*c rel {e_rc:.2e}")
    assert e_img < IMG_TOL and e_rc < IMG_TOL


def test_reconstruct_batched_series_with_prev(torch):
    """Batch of 3 frames from 3 turns, each regularised to (and started from) a
    different previous estimate; ragged sizes (J=5, K=7) on a 64-px grid."""
    N, J, K, U, M, C = 32, 5, 7, 3, 4, 8
    print_case("recon batched", N=N, J=J, K=K, U=U, M=M, C=C)
    ser = synth.real_time_series(seed=5, N=N, J=J, J_phys=8, K=K, U=U, frames=4)
    g = O.Geometry.make(N, J)
    plan = nl().Plan(N, J, K, U=U, batch=3, newton=M, cg=C)
    frames = [1, 2, 3]
    # previous estimates: oracle results of frames 0..2 started from scratch
    prevs = []
    for f in [0, 1, 2]:
        P = O.psf_kernel(ser.traj[f], g.R, g.G)
        prevs.append(O.reconstruct(g, O.grid(ser.y[f], ser.traj[f], g.R), P, newton=2, cg_iters=4))
    prevs = np.stack(prevs).astype(np.complex64)
    turns = [int(ser.turn[f]) for f in frames]
    z = plan.grid(dev(torch, ser.traj[frames]), dev(torch, ser.y[frames]), turns=turns)
    xp = dev(torch, prevs)
    x, img, _ = plan.reconstruct(z, turns, xprev=xp, init=2, want_img=True)
    x, img = host(x), host(img)
    for b, f in enumerate(frames):
        P = O.psf_kernel(ser.traj[f], g.R, g.G)
        xr = O.reconstruct(g, O.grid(ser.y[f], ser.traj[f], g.R), P, xprev=prevs[b], x0=prevs[b],
                           newton=M, cg_iters=C)
        e_img, e_rc = _recon_compare(g, x[b], img[b], xr)
        print(f"batched item {b}: image rel {e_img:.2e}  rho*c rel {e_rc:.2e}")
        assert e_img < IMG_TOL and e_rc < IMG_TOL


def test_reconstruct_is_deterministic(torch):
    s = synth.single_frame(seed=4, N=64, J=6, K=9)
    plan = nl().Plan(64, 6, 9, newton=3, cg=6)
    z = plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0])
    x1, _, _ = plan.reconstruct(z, [0])
    x2, _, _ = plan.reconstruct(z, [0])
    assert torch.equal(x1, x2)


def test_graph_replays_match_eager(torch):
    """Captured reconstructions (HIP graphs) replayed several times, with eager
    work and synchronisations in between, equal the uncaptured path bit for bit."""
    N, J, K, U = 64, 5, 9, 2
    ser = synth.real_time_series(seed=9, N=N, J=J, J_phys=6, K=K, U=U, frames=2)
    plan = nl().Plan(N, J, K, U=U, newton=3, cg=5)
    z0 = plan.grid(dev(torch, ser.traj[0:1]), dev(torch, ser.y[0:1]), turns=[0])
    z1 = plan.grid(dev(torch, ser.traj[1:2]), dev(torch, ser.y[1:2]), turns=[1])
    x0, img0, _ = plan.reconstruct(z0, [0], init=1, want_img=True)
    x1, img1, _ = plan.reconstruct(z1, [1], xprev=x0, init=2, want_img=True)
    ref0, ref1, refi = x0.clone(), x1.clone(), img1.clone()
    plan.set_graphs(True)
    a = torch.empty_like(ref0)
    bb = torch.empty_like(ref0)
    img = torch.empty_like(refi)
    for rep in range(3):
        a.fill_(float(rep))
        bb.zero_()
        torch.cuda.synchronize()
        plan.reconstruct(z0, [0], xhat=a, init=1)
        plan.reconstruct(z1, [1], xprev=a, xhat=bb, init=2, img=img)
        torch.cuda.synchronize()
        assert torch.equal(a, ref0) and torch.equal(bb, ref1) and torch.equal(img, refi), f"replay {rep}"
    plan.set_graphs(False)


def test_zero_data_is_a_fixed_point(torch):
    plan = nl().Plan(32, 3, 5, newton=3, cg=4)
    plan.psf(dev(torch, synth.radial_trajectory(32, 5, 64, 0, 1)), 0)
    z = torch.zeros(1, 3, 32, 32, dtype=torch.complex64, device="cuda")
    x, _, _ = plan.reconstruct(z, [0], init=1)
    g = O.Geometry.make(32, 3)
    assert np.array_equal(host(x)[0], g.initial().astype(np.complex64))


def test_state_and_argument_errors(torch):
    N = nl()
    plan = N.Plan(32, 3, 5, U=2)
    z = torch.zeros(1, 3, 32, 32, dtype=torch.complex64, device="cuda")
    with pytest.raises(N.NlinvError) as ei:
        plan.reconstruct(z, [1], init=1)          # PSF of turn 1 never computed
    assert ei.value.code == N.E_STATE
    with pytest.raises(N.NlinvError) as ei:
        plan.reconstruct(z, [2], init=1)          # turn out of range
    assert ei.value.code == N.E_ARG
    x = torch.zeros(1, plan.X, dtype=torch.complex64, device="cuda")
    plan.psf(dev(torch, synth.radial_trajectory(32, 5, 64, 0, 2)), 0)
    with pytest.raises(N.NlinvError) as ei:
        plan.reconstruct(z, [0], xprev=x, xhat=x, init=2)   # aliasing
    assert ei.value.code == N.E_ARG
    # the binding checks tensors before any library call: device, dtype, shape
    assert plan.device == torch.device("cuda", torch.cuda.current_device())
    with pytest.raises(ValueError):
        plan.reconstruct(z.cpu(), [0], init=1)
    with pytest.raises(TypeError):
        plan.reconstruct(z.to(torch.complex128), [0], init=1)
    with pytest.raises(ValueError):
        plan.reconstruct(z[:, :2].contiguous(), [0], init=1)
    with pytest.raises(ValueError):
        N.Plan(32, 3, 5, device="cpu")


# ---------------------------------------------------------------------------
# full-size real-time series (160 px, 10 virtual coils, 15 spokes x 320, 7 x 20)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c2_oracle():
    """Oracle reconstructions of frames 0 and 1 of the 160 px series (frame 1
    regularised to and started from frame 0); the series has 3 frames."""
    ser = synth.real_time_series(seed=2, frames=3)
    g = O.Geometry.make(160, 10)
    out, prev = [], None
    for f in range(2):
        P = O.psf_kernel(ser.traj[f], g.R, g.G)
        zr = O.grid(ser.y[f], ser.traj[f], g.R)
        prev = O.reconstruct(g, zr, P, xprev=prev, x0=prev, newton=7, cg_iters=20)
        out.append(prev)
    return ser, g, out


def _c2_errors(torch, c2_oracle, flags, cg_passes=0):
    ser, g, refs = c2_oracle
    plan = nl().Plan(160, 10, 15, U=5, newton=7, cg=20, flags=flags, cg_passes=cg_passes)
    x_prev_gpu, errs = None, []
    for f in range(2):
        t = int(ser.turn[f])
        z = plan.grid(dev(torch, ser.traj[f:f + 1]), dev(torch, ser.y[f:f + 1]), turns=[t])
        x, img, _ = plan.reconstruct(z, [t], xprev=x_prev_gpu, want_img=True)
        e_img, e_rc = _recon_compare(g, host(x)[0], host(img)[0], refs[f])
        print(f"c2 flags={flags} cg_passes={cg_passes} frame {f}: image rel {e_img:.2e}  rho*c rel {e_rc:.2e}",
              flush=True)
        errs.append((e_img, e_rc))
        x_prev_gpu = x.clone()
    return errs


@pytest.mark.parametrize("cg_passes", [6, 4])
def test_real_time_series_first_frames_c2(torch, c2_oracle, cg_passes):
    """160 px, 10 virtual coils, 15 spokes x 320, 7 x 20, frames 0 and 1 (full
    size), both forms of the CG iteration: within 1e-3 of the oracle."""
    print_case("recon c2 frames 0-1", N=160, J=10, K=15, M=7, C=20, cg_passes=cg_passes)
    for e_img, e_rc in _c2_errors(torch, c2_oracle, 0, cg_passes):
        assert e_img < IMG_TOL and e_rc < IMG_TOL


@pytest.mark.parametrize("cg_passes", [6, 4])
def test_relaxed_group_c2(torch, c2_oracle, cg_passes):
    """Full size, relaxed coupling with l = 0, o = 2: frame 0 strict, frames 1 and
    2 as one group from frame 0 (nlinv_reconstruct_frames, the bench's entry
    point).  Frame 1 heads the group, so its oracle result is the strict one;
    frame 2 takes M-1 steps from frame 0 and the last step towards frame 1."""
    print_case("relaxed group c2", N=160, J=10, K=15, M=7, C=20, l=0, o=2, cg_passes=cg_passes)
    ser, g, refs = c2_oracle
    P2 = O.psf_kernel(ser.traj[2], g.R, g.G)
    z2 = O.grid(ser.y[2], ser.traj[2], g.R)
    x = O.reconstruct(g, z2, P2, xprev=refs[0], x0=refs[0], newton=6, cg_iters=20)
    ref2 = x + O.newton_step(g, x, refs[1], z2, P2, O.alpha_schedule(7)[6], 20)
    plan = nl().Plan(160, 10, 15, U=5, batch=2, newton=7, cg=20, cg_passes=cg_passes)
    plan.set_batch(1)
    zs = [plan.grid(dev(torch, ser.traj[f:f + 1]), dev(torch, ser.y[f:f + 1]), turns=[int(ser.turn[f])])
          for f in range(3)]
    plan.set_batch(2)
    x0, i0, _ = plan.reconstruct_frames(zs[0], [int(ser.turn[0])], want_img=True)
    xg, ig, _ = plan.reconstruct_frames(torch.cat(zs[1:], 0), [int(t) for t in ser.turn[1:3]],
                                        xprev=x0[0], want_img=True)
    for f, (xf, imf, ref) in enumerate([(x0[0], i0[0], refs[0]), (xg[0], ig[0], refs[1]), (xg[1], ig[1], ref2)]):
        e_img, e_rc = _recon_compare(g, host(xf), host(imf), ref)
        print(f"relaxed c2 frame {f}: image rel {e_img:.2e}  rho*c rel {e_rc:.2e}", flush=True)
        assert e_img < IMG_TOL and e_rc < IMG_TOL


@pytest.mark.parametrize("cg_passes", [6, 4])
def test_batched_items_equal_plain_c2(torch, c2_oracle, cg_passes):
    """Full size, batched launch configuration: every item of a batch-16 plan
    reconstructs exactly (bit for bit) what the batch-1 plan does on the same
    gridded data, so the batch-1 oracle parity carries over to each item."""
    print_case("batched c2 items", N=160, J=10, K=15, M=7, C=20, B=16, cg_passes=cg_passes)
    ser, g, refs = c2_oracle
    one = nl().Plan(160, 10, 15, U=5, newton=7, cg=20, cg_passes=cg_passes)
    t = int(ser.turn[0])
    z = one.grid(dev(torch, ser.traj[0:1]), dev(torch, ser.y[0:1]), turns=[t])
    x1, i1, _ = one.reconstruct(z, [t], want_img=True)
    many = nl().Plan(160, 10, 15, U=5, batch=16, newton=7, cg=20, cg_passes=cg_passes)
    many.psf(dev(torch, ser.traj[0]), t)
    zb = z.expand(16, -1, -1, -1).contiguous()
    xb, ib, _ = many.reconstruct(zb, [t] * 16, want_img=True)
    for b in (0, 7, 15):
        assert torch.equal(xb[b], x1[0]) and torch.equal(ib[b], i1[0]), b


def test_batched_items_equal_plain_past_the_infinity_cache(torch, c2_oracle):
    """A batch whose half-transformed grid (36 x 10 x 320 x 160 x 16 B = 295 MB)
    exceeds the 256 MiB Infinity Cache runs its column passes in the other
    block order (tile fastest instead of channel fastest); its items still
    reconstruct the batch-1 plan's bits."""
    B = 36
    print_case("batched c2 items past the cache", N=160, J=10, K=15, M=7, C=20, B=B, cg_passes=6)
    assert B * 10 * 320 * 160 * 16 > 256 << 20
    ser, g, refs = c2_oracle
    one = nl().Plan(160, 10, 15, U=5, newton=7, cg=20, cg_passes=6)
    t = int(ser.turn[0])
    z = one.grid(dev(torch, ser.traj[0:1]), dev(torch, ser.y[0:1]), turns=[t])
    x1, i1, _ = one.reconstruct(z, [t], want_img=True)
    many = nl().Plan(160, 10, 15, U=5, batch=B, newton=7, cg=20, cg_passes=6)
    many.psf(dev(torch, ser.traj[0]), t)
    zb = z.expand(B, -1, -1, -1).contiguous()
    xb, ib, _ = many.reconstruct(zb, [t] * B, want_img=True)
    for b in (0, 17, B - 1):
        assert torch.equal(xb[b], x1[0]) and torch.equal(ib[b], i1[0]), b


def test_check_finite_flag(torch):
    """NLINV_F_CHECK_FINITE: a clean reconstruction syncs fine; a non-finite
    input sample makes the next nlinv_sync report NLINV_E_NONFINITE once (the
    flag is cleared by the report); without the flag nothing is checked."""
    N, J, K = 32, 3, 5
    print_case("check finite", N=N, J=J, K=K)
    s = synth.single_frame(seed=9, N=N, J=J, K=K)
    lib = nl()
    plan = lib.Plan(N, J, K, newton=2, cg=3, flags=lib.F_CHECK_FINITE)
    z = plan.grid(dev(torch, s.traj), dev(torch, s.y), turns=[0])
    plan.reconstruct(z, [0])
    plan.sync()
    bad = z.clone()
    bad[0, 1, 5, 7] = complex(float("nan"), 0.0)
    plan.reconstruct(bad, [0])
    with pytest.raises(lib.NlinvError) as ei:
        plan.sync()
    assert ei.value.code == lib.E_NONFINITE
    plan.sync()                                   # reported once, then cleared
    x, _, _ = plan.reconstruct(z, [0])
    plan.sync()
    assert bool(torch.isfinite(torch.view_as_real(x)).all())
    plain = lib.Plan(N, J, K, newton=2, cg=3)
    plain.psf(dev(torch, s.traj[0]), 0)
    xb, _, _ = plain.reconstruct(bad, [0])
    plain.sync()
    assert not bool(torch.isfinite(torch.view_as_real(xb)).all())
