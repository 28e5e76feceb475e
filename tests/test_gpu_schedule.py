"""Tile schedules of the CG column passes (columns per block, 8 or 4): the
decomposition changes which block computes a column, not the arithmetic of
any column, so reconstructions and operator applications agree bit for bit,
and with the oracle to the usual bars."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()
    return _t


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("N,J,K,B,G,flags", [(64, 8, 13, 3, 0, 0), (160, 10, 15, 1, 0, 0), (120, 3, 9, 2, 480, 0),
                                             (64, 8, 13, 2, 0, 2)])    # exact gridding
def test_column_tiles_agree_bit_for_bit(torch, N, J, K, B, G, flags):
    from paper_1701_08361_amd import nlinv as nl
    print(f"[case] column tiles N={N} J={J} K={K} B={B} G={G} flags={flags}", flush=True)
    s = [synth.single_frame(seed=20 + b, N=N, J=J, K=K) for b in range(B)]
    traj = torch.from_numpy(np.concatenate([f.traj for f in s])).cuda()
    y = torch.from_numpy(np.concatenate([f.y for f in s])).cuda()
    out = {}
    for tile in (0, 4, 8):
        plan = nl.Plan(N, J, K, batch=B, newton=3, cg=6, G=G, col_tile=tile, flags=flags)
        z = plan.grid(traj, y, turns=[0] * B) if B == 1 else None
        if B > 1:
            plan.psf(traj[0].contiguous(), 0)
            z = plan.grid(traj, y)
        x, img, _ = plan.reconstruct(z, [0] * B, want_img=True)
        p = torch.from_numpy(np.stack([synth.random_xhat(5 + b, plan.R, J, plan.Gc) for b in range(B)])).cuda()
        q = plan.apply_normal([0] * B, x, p, 0.25)
        torch.cuda.synchronize()
        out[tile] = (x.cpu().numpy(), img.cpu().numpy(), q.cpu().numpy(), plan)
    for tile in (4, 8):
        for a, b in zip(out[0][:3], out[tile][:3]):
            assert np.array_equal(a, b), f"col_tile={tile} differs from the default"
    # and the default against the oracle (first item)
    plan = out[0][3]
    g = O.Geometry.make(N, J, plan.G)
    P = O.psf_kernel(s[0].traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(s[0].y[0], s[0].traj[0], g.R), P, newton=3, cg_iters=6)
    e = rel(out[0][1][0], O.image(g, xr))
    print(f"image rel {e:.2e}")
    assert e < 1e-3
    for t in out.values():
        t[3].close()


def test_psf_of_all_samples_equals_psf(torch):
    """nlinv_psf_samples with every sample builds the same PSF kernel and
    gridding table as nlinv_psf: the reconstructions agree bit for bit."""
    from paper_1701_08361_amd import nlinv as nl
    N, J, K = 64, 4, 9
    print(f"[case] psf samples = K * S_r N={N} J={J} K={K}", flush=True)
    s = synth.single_frame(seed=31, N=N, J=J, K=K)
    traj = torch.from_numpy(s.traj).cuda()
    y = torch.from_numpy(s.y).cuda()
    res = []
    for samples in (None, K * 2 * N):
        plan = nl.Plan(N, J, K, newton=2, cg=4)
        plan.psf(traj[0].contiguous(), 0, samples=samples)
        z = plan.grid(traj, y, turns=[0])
        x, img, _ = plan.reconstruct(z, [0], want_img=True)
        torch.cuda.synchronize()
        res.append((z.cpu(), x.cpu(), img.cpu()))
        plan.close()
    for a, b in zip(*res):
        assert torch.equal(a, b)


@pytest.mark.parametrize("N,J,K,B,seed", [(64, 8, 13, 3, 40), (128, 5, 11, 2, 44), (32, 3, 5, 1, 46)])
def test_cg_forms_match_oracle(torch, N, J, K, B, seed):
    """The four-pass CG iteration (direction update, W^-1 p and the vector step
    folded into the operator's passes, Re<p, q> from the spectrum) and the
    six-pass one: each item within 1e-3 of the oracle, and the two forms within
    1e-4 of each other (the same CG up to rounding).  Four-pass results do not
    depend on the tile schedule (bit for bit)."""
    from paper_1701_08361_amd import nlinv as nl
    M, C = 4, 8
    print(f"[case] cg forms N={N} J={J} K={K} B={B} M={M} C={C}", flush=True)
    s = [synth.single_frame(seed=seed + b, N=N, J=J, K=K) for b in range(B)]
    traj = torch.from_numpy(np.concatenate([f.traj for f in s])).cuda()
    y = torch.from_numpy(np.concatenate([f.y for f in s])).cuda()
    imgs = {}
    for passes, tile in ((6, 0), (4, 0), (4, 4)):
        plan = nl.Plan(N, J, K, batch=B, newton=M, cg=C, cg_passes=passes, col_tile=tile)
        plan.psf(traj[0].contiguous(), 0)
        z = plan.grid(traj, y)
        _, img, _ = plan.reconstruct(z, [0] * B, want_img=True)
        torch.cuda.synchronize()
        imgs[(passes, tile)] = img.cpu().numpy()
        plan.close()
    assert np.array_equal(imgs[(4, 0)], imgs[(4, 4)])
    g = O.Geometry.make(N, J)
    P = O.psf_kernel(s[0].traj[0], g.R, g.G)
    for b in range(B):
        assert np.array_equal(s[b].traj, s[0].traj)      # one trajectory (turn 0) for every item
        xr = O.reconstruct(g, O.grid(s[b].y[0], s[0].traj[0], g.R), P, newton=M, cg_iters=C)
        ref = O.image(g, xr)
        e6, e4 = rel(imgs[(6, 0)][b], ref), rel(imgs[(4, 0)][b], ref)
        d = rel(imgs[(4, 0)][b], imgs[(6, 0)][b])
        print(f"item {b}: six-pass rel {e6:.2e}, four-pass rel {e4:.2e}, between forms {d:.2e}")
        assert e6 < 1e-3 and e4 < 1e-3 and d < 1e-4


@pytest.mark.parametrize("N,J,K,G", [(32, 2, 5, 0), (64, 4, 9, 0), (128, 3, 9, 0), (160, 4, 9, 0), (192, 3, 9, 0),
                                     (216, 2, 9, 0), (224, 2, 9, 0), (240, 2, 9, 0), (256, 2, 9, 0)])
def test_toeplitz_factorisations_match_oracle(torch, N, J, K, G):
    """The alternative factorisation of the Toeplitz row pass (fft_split = 1;
    every grid side): the CG operator against the oracle at the operator bar,
    and a short reconstruction in both CG forms against the oracle at the
    image bar."""
    from paper_1701_08361_amd import nlinv as nl
    print(f"[case] fft split N={N} J={J} K={K}", flush=True)
    s = synth.single_frame(seed=41, N=N, J=J, K=K)
    traj = torch.from_numpy(s.traj).cuda()
    y = torch.from_numpy(s.y).cuda()
    g = O.Geometry.make(N, J)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    x0 = synth.random_xhat(42, g.R, J, g.Gc, 1.0, 0.3)
    p = synth.random_xhat(43, g.R, J, g.Gc, 1.0, 0.3)
    ref_q = O.normal(g, x0.astype(np.complex128), p.astype(np.complex128), P) + 0.2 * p
    xr = O.reconstruct(g, O.grid(s.y[0], s.traj[0], g.R), P, newton=2, cg_iters=4)
    for passes in (6, 4):
        plan = nl.Plan(N, J, K, newton=2, cg=4, fft_split=1, cg_passes=passes)
        z = plan.grid(traj, y, turns=[0])
        q = plan.apply_normal([0], torch.from_numpy(x0[None]).cuda(), torch.from_numpy(p[None]).cuda(), 0.2)
        x, img, _ = plan.reconstruct(z, [0], want_img=True)
        e_q = rel(q.cpu().numpy()[0], ref_q)
        e_i = rel(img.cpu().numpy()[0], O.image(g, xr))
        print(f"fft_split 1, {passes} passes: operator rel {e_q:.2e}, image rel {e_i:.2e}")
        assert e_q < 1e-4 and e_i < 1e-3
        plan.close()
