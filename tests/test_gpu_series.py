"""Frame series on the GPU: the relaxed temporal coupling (Sec. 3.3, temporal
decomposition, equation for h(n, m)) through nlinv_reconstruct_frames, and
partial batches through nlinv_set_batch, against the FP64 oracle and against
the plain entry points.
"""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

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


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _grid_all(torch, plan, ser, frames):
    """z [F][J][R][R] of the given frames, one gridding call per frame (batch 1)."""
    out = []
    plan.set_batch(1)
    for f in frames:
        out.append(plan.grid(dev(torch, ser.traj[f:f + 1]), dev(torch, ser.y[f:f + 1]), turns=[int(ser.turn[f])]))
    plan.set_batch(plan.Bmax)
    return torch.cat(out, 0)


def test_frames_count1_equals_reconstruct(torch):
    """count = 1 is the strict order: bit-identical to nlinv_reconstruct."""
    N, J, K, U, M, C = 32, 4, 7, 2, 3, 6
    print_case("frames count=1", N=N, J=J, K=K, M=M, C=C)
    ser = synth.real_time_series(seed=21, N=N, J=J, J_phys=6, K=K, U=U, frames=2)
    plan = nl().Plan(N, J, K, U=U, batch=3, newton=M, cg=C)
    z = _grid_all(torch, plan, ser, [0, 1])
    plan.set_batch(1)
    x0, img0, _ = plan.reconstruct(z[0:1], [0], init=1, want_img=True)
    x1, img1, _ = plan.reconstruct(z[1:2], [1], xprev=x0, init=2, want_img=True)
    plan.set_batch(3)
    for graphs in (False, True):
        plan.set_graphs(graphs)
        for rep in range(2 if graphs else 1):
            f0, i0, _ = plan.reconstruct_frames(z[0:1], [0], xprev=None, want_img=True)
            f1, i1, _ = plan.reconstruct_frames(z[1:2], [1], xprev=f0[0], want_img=True)
            torch.cuda.synchronize()
            assert torch.equal(f0, x0) and torch.equal(f1, x1), (graphs, rep)
            assert torch.equal(i0, img0) and torch.equal(i1, img1), (graphs, rep)
    plan.set_graphs(False)
    assert plan.B == 3


@pytest.mark.parametrize("M,l,o,passes", [(3, 2, 3, 6), (1, 0, 2, 6), (2, 1, 4, 6), (3, 2, 3, 4)])
def test_relaxed_series_matches_oracle(torch, M, l, o, passes):
    """A 9-frame series under h(n, m) with groups of o frames: every frame's
    image and coil images match the oracle's relaxed schedule (both CG
    iteration forms)."""
    N, J, K, U, C, F = 32, 5, 7, 3, 8, 9
    print_case("relaxed series", N=N, J=J, K=K, U=U, M=M, C=C, F=F, l=l, o=o, passes=passes)
    ser = synth.real_time_series(seed=23, N=N, J=J, J_phys=8, K=K, U=U, frames=F)
    g = O.Geometry.make(N, J)
    src = O.relaxed_sources(F, l, o)
    zs = [O.grid(ser.y[f], ser.traj[f], g.R) for f in range(F)]
    Ps = [O.psf_kernel(ser.traj[f], g.R, g.G) for f in range(F)]
    ref = O.reconstruct_series(g, zs, Ps, src, newton=M, cg_iters=C)

    plan = nl().Plan(N, J, K, U=U, batch=o, newton=M, cg=C, cg_passes=passes)
    z = _grid_all(torch, plan, ser, range(F))
    X = plan.X
    xs = torch.empty(F, X, dtype=torch.complex64, device="cuda")
    imgs = torch.empty(F, N, N, dtype=torch.float32, device="cuda")
    n = 0
    while n < F:
        # a group: frames sharing one source (strict frames are groups of one)
        k = 1
        while n + k < F and src[n + k] == src[n] and n > l:
            k += 1
        prev = xs[n - 1] if n > 0 else None
        assert src[n] == n - 1
        plan.reconstruct_frames(z[n:n + k], [int(t) for t in ser.turn[n:n + k]], xprev=prev,
                                xhat=xs[n:n + k], img=imgs[n:n + k])
        n += k
    xs, imgs = host(xs), host(imgs)
    worst = 0.0
    for f in range(F):
        e_img = rel(imgs[f], O.image(g, ref[f]))
        e_rc = rel(O.coil_images(g, xs[f].astype(np.complex128)), O.coil_images(g, ref[f]))
        worst = max(worst, e_img, e_rc)
        assert e_img < IMG_TOL and e_rc < IMG_TOL, (f, e_img, e_rc)
    print(f"relaxed series M={M} l={l} o={o}: worst rel {worst:.2e}")


def test_set_batch_partial_equals_smaller_plan(torch):
    """A batch-4 plan restricted to 2 items grids and reconstructs exactly like a
    batch-2 plan."""
    N, J, K, U, M, C = 32, 3, 5, 2, 2, 5
    print_case("set_batch", N=N, J=J, K=K, M=M, C=C)
    ser = synth.real_time_series(seed=25, N=N, J=J, J_phys=4, K=K, U=U, frames=2)
    big = nl().Plan(N, J, K, U=U, batch=4, newton=M, cg=C)
    small = nl().Plan(N, J, K, U=U, batch=2, newton=M, cg=C)
    big.set_batch(2)
    turns = [int(t) for t in ser.turn[:2]]
    traj, y = dev(torch, ser.traj[:2]), dev(torch, ser.y[:2])
    zb = big.grid(traj, y, turns=turns)
    zs = small.grid(traj, y, turns=turns)
    assert torch.equal(zb, zs)
    xb, ib, _ = big.reconstruct(zb, turns, init=1, want_img=True)
    xs, is_, _ = small.reconstruct(zs, turns, init=1, want_img=True)
    assert torch.equal(xb, xs) and torch.equal(ib, is_)


def test_frames_argument_errors(torch):
    N = nl()
    plan = N.Plan(32, 3, 5, U=1, batch=2)
    plan.psf(dev(torch, synth.radial_trajectory(32, 5, 64, 0, 1)), 0)
    z = torch.zeros(3, 3, 32, 32, dtype=torch.complex64, device="cuda")
    with pytest.raises(N.NlinvError) as ei:
        plan.reconstruct_frames(z, [0, 0, 0])                 # count > batch
    assert ei.value.code == N.E_ARG
    x = torch.zeros(2, plan.X, dtype=torch.complex64, device="cuda")
    with pytest.raises(N.NlinvError) as ei:
        plan.reconstruct_frames(z[:2], [0, 0], xprev=x[1], xhat=x)   # overlap
    assert ei.value.code == N.E_ARG
    with pytest.raises(N.NlinvError) as ei:
        plan.set_batch(3)
    assert ei.value.code == N.E_ARG
    assert plan.B == 2


def test_uneven_channel_counts_share_a_batch(torch):
    """Series with fewer coils join a batched plan of more channels with their
    missing channels zero: a channel with zero data and a zero coil spectrum
    keeps a zero residual, right-hand side, CG direction and update, so it
    stays exactly zero and only appends exact zeros to every channel sum and
    partial-sum array (the real channels' block assignment and summation
    order do not change).  So the padded item equals its own smaller plan bit
    for bit, and the full item its batch-1 plan."""
    N, K, U, M, C = 32, 5, 2, 3, 6
    Ja, Jb = 6, 10
    print_case("uneven channels", N=N, Ja=Ja, Jb=Jb, K=K, M=M, C=C)
    sa = synth.real_time_series(seed=27, N=N, J=Ja, J_phys=8, K=K, U=U, frames=2)
    sb = synth.real_time_series(seed=28, N=N, J=Jb, J_phys=12, K=K, U=U, frames=2)
    pa = nl().Plan(N, Ja, K, U=U, newton=M, cg=C)
    pb = nl().Plan(N, Jb, K, U=U, newton=M, cg=C)
    both = nl().Plan(N, Jb, K, U=U, batch=2, newton=M, cg=C)
    za = [pa.grid(dev(torch, sa.traj[f:f + 1]), dev(torch, sa.y[f:f + 1]), turns=[int(sa.turn[f])]) for f in range(2)]
    zb = [pb.grid(dev(torch, sb.traj[f:f + 1]), dev(torch, sb.y[f:f + 1]), turns=[int(sb.turn[f])]) for f in range(2)]
    for t in range(U):                 # the batch plan needs the turns' PSF kernels
        both.psf(dev(torch, sa.traj[t]), t)
    assert [int(t) for t in sa.turn[:2]] == [int(t) for t in sb.turn[:2]]
    R2, gc2 = N * N, both.Gc * both.Gc
    assert both.X == R2 + Jb * gc2
    xa = xb = x2 = None
    for f in range(2):
        ts = [int(sa.turn[f])]
        xa, ia, _ = pa.reconstruct(za[f], ts, xprev=xa, init=1 if f == 0 else 2, want_img=True)
        xb, ib, _ = pb.reconstruct(zb[f], ts, xprev=xb, init=1 if f == 0 else 2, want_img=True)
        z2 = torch.zeros(2, Jb, N, N, dtype=torch.complex64, device="cuda")
        z2[0, :Ja] = za[f][0]
        z2[1] = zb[f][0]
        x2, i2, _ = both.reconstruct(z2, ts * 2, xprev=x2, init=1 if f == 0 else 2, want_img=True)
        # the padded item: its extra coil blocks stay exactly zero
        assert torch.count_nonzero(x2[0, R2 + Ja * gc2:]) == 0
        assert torch.equal(x2[0, :R2 + Ja * gc2], xa[0]) and torch.equal(i2[0], ia[0]), f
        # the full item is untouched by its neighbour
        assert torch.equal(x2[1], xb[0]) and torch.equal(i2[1], ib[0])


def test_uneven_spoke_counts_share_a_batch(torch):
    """A turn declared with fewer spokes (nlinv_psf_spokes) builds its PSF
    kernel and gridding table from those spokes alone; a series with 9
    spokes per frame then runs in a 15-spoke batched plan, its data padded
    with spokes that are never read, and equals its own 9-spoke plan bit for
    bit, while the 15-spoke item equals its batch-1 plan."""
    N, J, U, M, C = 32, 4, 2, 3, 5
    Ka, Kb = 9, 15
    print_case("uneven spokes", N=N, J=J, Ka=Ka, Kb=Kb, M=M, C=C)
    sa = synth.real_time_series(seed=41, N=N, J=J, J_phys=6, K=Ka, U=U, frames=2)
    sb = synth.real_time_series(seed=42, N=N, J=J, J_phys=6, K=Kb, U=U, frames=2)
    Sr = 2 * N
    pa = nl().Plan(N, J, Ka, U=U, newton=M, cg=C)
    pb = nl().Plan(N, J, Kb, U=U, newton=M, cg=C)
    both = nl().Plan(N, J, Kb, U=2 * U, batch=2, newton=M, cg=C)   # turns 0..U-1: a, U..2U-1: b
    # a's trajectories and data padded to Kb spokes (zeros, never read)
    ta = np.zeros((2, Kb, Sr, 2), np.float32)
    ta[:, :Ka] = sa.traj
    ya = np.zeros((2, J, Kb * Sr), np.complex64)
    ya[:, :, :Ka * Sr] = sa.y
    for t in range(U):
        both.psf(dev(torch, ta[t]), t, spokes=Ka)
        both.psf(dev(torch, sb.traj[t]), U + t)
    with pytest.raises(nl().NlinvError):
        both.psf(dev(torch, ta[0]), 0, spokes=Kb + 1)
    xa = xb = x2 = None
    for f in range(2):
        t = int(sa.turn[f])
        assert t == int(sb.turn[f])
        za = pa.grid(dev(torch, sa.traj[f:f + 1]), dev(torch, sa.y[f:f + 1]), turns=[t])
        zb = pb.grid(dev(torch, sb.traj[f:f + 1]), dev(torch, sb.y[f:f + 1]), turns=[t])
        traj2 = dev(torch, np.stack([ta[f], sb.traj[f]]))
        y2 = dev(torch, np.stack([ya[f], sb.y[f]]))
        z2 = both.grid(traj2, y2, turns=[t, U + t])
        assert torch.equal(z2[0], za[0]) and torch.equal(z2[1], zb[0])
        xa, ia, _ = pa.reconstruct(za, [t], xprev=xa, init=1 if f == 0 else 2, want_img=True)
        xb, ib, _ = pb.reconstruct(zb, [t], xprev=xb, init=1 if f == 0 else 2, want_img=True)
        x2, i2, _ = both.reconstruct(z2, [t, U + t], xprev=x2, init=1 if f == 0 else 2, want_img=True)
        assert torch.equal(x2[0], xa[0]) and torch.equal(i2[0], ia[0]), f
        assert torch.equal(x2[1], xb[0]) and torch.equal(i2[1], ib[0]), f


def test_uneven_resolutions_share_a_batch(torch):
    """Image sides, coil counts and spoke counts all uneven in one launch: a
    48 px, 3-coil, 7-spoke series runs on the 128 grid of a 64 px, 4-coil,
    9-spoke batched plan (gamma = 4/3 for it, Sec. 3.2), its 7 x 96 samples
    packed at the start of the plan's 9 x 128 layout (nlinv_psf_samples) and
    its fourth channel zero.  It equals its own 48 px plan on the 128 grid bit
    for bit (image, coil spectra; the extra channel stays exactly zero), and
    the 64 px item equals its batch-1 plan."""
    U, M, C = 2, 3, 5
    (Na, Ja, Ka), (Nb, Jb, Kb) = (48, 3, 7), (64, 4, 9)
    G = 2 * Nb
    print_case("uneven resolutions", Na=Na, Ja=Ja, Ka=Ka, Nb=Nb, Jb=Jb, Kb=Kb, G=G, M=M, C=C)
    sa = synth.real_time_series(seed=43, N=Na, J=Ja, J_phys=6, K=Ka, U=U, frames=2)
    sb = synth.real_time_series(seed=44, N=Nb, J=Jb, J_phys=6, K=Kb, U=U, frames=2)
    na, S = Ka * 2 * Na, Kb * 2 * Nb
    pa = nl().Plan(Na, Ja, Ka, G=G, U=U, newton=M, cg=C)
    pb = nl().Plan(Nb, Jb, Kb, U=U, newton=M, cg=C)
    both = nl().Plan(Nb, Jb, Kb, U=2 * U, batch=2, newton=M, cg=C)   # turns 0..U-1: a, U..2U-1: b
    assert (pa.R, pa.G) == (both.R, both.G)
    ta = np.zeros((2, S, 2), np.float32)
    ta[:, :na] = sa.traj.reshape(2, na, 2)
    ta = ta.reshape(2, Kb, 2 * Nb, 2)
    ya = np.zeros((2, Jb, S), np.complex64)
    ya[:, :Ja, :na] = sa.y
    for t in range(U):
        both.psf(dev(torch, ta[t]), t, samples=na)
        both.psf(dev(torch, sb.traj[t]), U + t)
    with pytest.raises(nl().NlinvError):
        both.psf(dev(torch, ta[0]), 0, samples=S + 1)
    Xa = pa.X
    xa = xb = x2 = None
    for f in range(2):
        t = int(sa.turn[f])
        assert t == int(sb.turn[f])
        za = pa.grid(dev(torch, sa.traj[f:f + 1]), dev(torch, sa.y[f:f + 1]), turns=[t])
        zb = pb.grid(dev(torch, sb.traj[f:f + 1]), dev(torch, sb.y[f:f + 1]), turns=[t])
        z2 = both.grid(dev(torch, np.stack([ta[f], sb.traj[f]])), dev(torch, np.stack([ya[f], sb.y[f]])),
                       turns=[t, U + t])
        assert torch.equal(z2[0, :Ja], za[0]) and not torch.any(z2[0, Ja:] != 0)
        assert torch.equal(z2[1], zb[0])
        xa, ia, _ = pa.reconstruct(za, [t], xprev=xa, init=1 if f == 0 else 2, want_img=True)
        xb, ib, _ = pb.reconstruct(zb, [t], xprev=xb, init=1 if f == 0 else 2, want_img=True)
        x2, i2, _ = both.reconstruct(z2, [t, U + t], xprev=x2, init=1 if f == 0 else 2, want_img=True)
        assert torch.equal(x2[0, :Xa], xa[0]) and not torch.any(x2[0, Xa:] != 0), f
        assert torch.equal(i2[0], ia[0]) and torch.equal(pa.crop(i2[0]), pa.crop(ia[0])), f
        assert torch.equal(x2[1], xb[0]) and torch.equal(i2[1], ib[0]), f
    print("uneven resolutions: bit for bit")


def test_relaxed_group_side_by_side_graphs_match_eager(torch):
    """A relaxed group of three frames in the four-pass form (its shared Newton
    steps as one chain per member on streams of their own, forked from and
    joined back into the plan's stream) gives the same bits eagerly and as a
    captured graph, over replays with eager runs of the group in between, and
    matches the oracle's relaxed schedule."""
    N, J, K, U, M, C = 32, 4, 7, 3, 3, 5
    print_case("relaxed group side by side, graphs", N=N, J=J, K=K, U=U, M=M, C=C)
    ser = synth.real_time_series(seed=23, N=N, J=J, J_phys=6, K=K, U=U, frames=4)
    plan = nl().Plan(N, J, K, U=U, batch=3, newton=M, cg=C, cg_passes=4)
    z = _grid_all(torch, plan, ser, range(4))
    plan.set_batch(1)
    x0, _, _ = plan.reconstruct(z[0:1], [int(ser.turn[0])], init=1)
    plan.set_batch(3)
    turns = [int(t) for t in ser.turn[1:4]]
    ref, refi, _ = plan.reconstruct_frames(z[1:4], turns, xprev=x0[0], want_img=True)
    torch.cuda.synchronize()
    ref, refi = ref.clone(), refi.clone()
    for rep in range(3):
        plan.set_graphs(True)
        f, i, _ = plan.reconstruct_frames(z[1:4], turns, xprev=x0[0], want_img=True)
        torch.cuda.synchronize()
        assert torch.equal(f, ref) and torch.equal(i, refi), rep
        plan.set_graphs(False)
        f, _, _ = plan.reconstruct_frames(z[1:4], turns, xprev=x0[0])
        torch.cuda.synchronize()
        assert torch.equal(f, ref), rep
    # the oracle's relaxed schedule: frame 0 strict, frames 1..3 one group
    g = O.Geometry.make(N, J)
    Ps = [O.psf_kernel(ser.traj[f], g.R, g.G) for f in range(4)]
    zs = [O.grid(ser.y[f], ser.traj[f], g.R) for f in range(4)]
    xo = O.reconstruct_series(g, zs, Ps, O.relaxed_sources(4, 0, 3), newton=M, cg_iters=C)
    imgs = host(refi)
    worst = max(rel(imgs[k], O.image(g, xo[k + 1])) for k in range(3))
    print(f"relaxed group side by side: graphs equal eager; worst image rel vs oracle {worst:.2e}")
    assert worst < IMG_TOL
