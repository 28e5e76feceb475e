"""Channel compression on the GPU (Sec. 3.1, preprocessing): the compression
product and its calibration against the oracle, and the whole preprocessing
plus reconstruction from receive-channel data."""
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
    nlinv.load()            # fails loudly when the HIP library is missing
    return _t


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("N,J,Jp,K,B", [(32, 4, 9, 5, 2), (64, 8, 30, 13, 3), (160, 10, 64, 15, 1)])
def test_compress_matches_oracle(torch, N, J, Jp, K, B):
    from paper_1701_08361_amd import nlinv
    print(f"[case] compress N={N} J={J} Jp={Jp} K={K} B={B}", flush=True)
    plan = nlinv.Plan(N, J, K, batch=B)
    rng = np.random.default_rng(N + Jp)
    cc = (rng.standard_normal((J, Jp)) + 1j * rng.standard_normal((J, Jp))).astype(np.complex64)
    yp = (rng.standard_normal((B, Jp, plan.S)) + 1j * rng.standard_normal((B, Jp, plan.S))).astype(np.complex64)
    y = plan.compress(torch.from_numpy(cc).cuda(), torch.from_numpy(yp).cuda()).cpu().numpy()
    e = rel(y, O.compress(cc, yp))
    print(f"compress rel {e:.2e}")
    assert e < 1e-6


@pytest.mark.parametrize("N,J,Jp,K", [(32, 4, 9, 5), (160, 10, 30, 15), (64, 16, 64, 13),
                                      (32, 8, 128, 5)])     # the most receive channels
def test_compression_matrix_matches_oracle(torch, N, J, Jp, K):
    """Calibration on one receive-channel frame: orthonormal rows spanning the
    oracle's principal subspace (compared as projectors, rows being defined up
    to a phase)."""
    from paper_1701_08361_amd import nlinv
    print(f"[case] calibration N={N} J={J} Jp={Jp} K={K}", flush=True)
    ser = synth.real_time_series(seed=81, N=N, J=J, J_phys=Jp, K=K, U=1, frames=1, compress=False)
    plan = nlinv.Plan(N, J, K)
    cc = plan.compression_matrix(torch.from_numpy(ser.y[0]).cuda()).cpu().numpy().astype(np.complex128)
    ref = O.compression_matrix(ser.y[0], J)
    e = rel(cc.conj().T @ cc, ref.conj().T @ ref)
    orth = np.abs(cc @ cc.conj().T - np.eye(J)).max()
    print(f"projector rel {e:.2e}, orthonormality {orth:.1e}")
    assert e < 1e-5 and orth < 1e-5


def test_preprocessing_and_reconstruction_from_receive_channels(torch):
    """Receive channels -> calibration + compression -> gridding ->
    reconstruction on the GPU, against the oracle doing the same steps (the
    image is independent of the phase left free in each compression row)."""
    from paper_1701_08361_amd import nlinv
    N, J, Jp, K, M, C = 64, 6, 20, 13, 4, 8
    print(f"[case] receive channels N={N} J={J} Jp={Jp} K={K} M={M} C={C}", flush=True)
    ser = synth.real_time_series(seed=83, N=N, J=J, J_phys=Jp, K=K, U=1, frames=1, compress=False)
    plan = nlinv.Plan(N, J, K, newton=M, cg=C)
    yp = torch.from_numpy(ser.y).cuda()                     # [1, Jp, S]
    cc = plan.compression_matrix(yp[0])
    y = plan.compress(cc, yp)
    z = plan.grid(torch.from_numpy(ser.traj).cuda(), y, turns=[0])
    x, img, _ = plan.reconstruct(z, [0], want_img=True)
    g = O.Geometry.make(N, J)
    ccr = O.compression_matrix(ser.y[0], J)
    yr = O.compress(ccr, ser.y[0])
    P = O.psf_kernel(ser.traj[0], g.R, g.G)
    xr = O.reconstruct(g, O.grid(yr, ser.traj[0], g.R), P, newton=M, cg_iters=C)
    e = rel(img.cpu().numpy()[0], O.image(g, xr))
    print(f"receive-channel pipeline image rel {e:.2e}")
    assert e < 1e-3
