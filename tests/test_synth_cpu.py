"""The seeded input generator shared by the oracle and the GPU tests: it is
deterministic, and its trajectories and scaling follow the readings of the
paper's acquisition (Fig. reorder: spokes 2 pi / K apart, turns offset by
2 pi / (K U); twofold readout oversampling; data scaled to norm 100, then
complex noise)."""
import numpy as np
import pytest

from paper_1701_08361_amd import synth


def test_same_seed_same_data_other_seed_other_data():
    a = synth.single_frame(seed=5, N=16, J=3, K=5)
    b = synth.single_frame(seed=5, N=16, J=3, K=5)
    c = synth.single_frame(seed=6, N=16, J=3, K=5)
    for f in ("traj", "y", "truth", "coils"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert not np.array_equal(a.y, c.y)
    s1 = synth.real_time_series(seed=3, N=16, J=3, J_phys=5, K=5, U=3, frames=4)
    s2 = synth.real_time_series(seed=3, N=16, J=3, J_phys=5, K=5, U=3, frames=4)
    assert np.array_equal(s1.y, s2.y) and np.array_equal(s1.traj, s2.traj)


def test_series_shapes_types_and_turns():
    N, J, Jp, K, U, F = 16, 3, 5, 5, 3, 4
    s = synth.real_time_series(seed=3, N=N, J=J, J_phys=Jp, K=K, U=U, frames=F)
    assert s.traj.shape == (F, K, 2 * N, 2) and s.traj.dtype == np.float32
    assert s.y.shape == (F, J, K * 2 * N) and s.y.dtype == np.complex64
    assert list(s.turn) == [n % U for n in range(F)]
    raw = synth.real_time_series(seed=3, N=N, J=J, J_phys=Jp, K=K, U=U, frames=F, compress=False)
    assert raw.y.shape == (F, Jp, K * 2 * N)


def test_trajectory_angles_and_readout():
    N, K, U = 16, 7, 3
    S_r = 2 * N
    for turn in range(U):
        t = synth.radial_trajectory(N, K, S_r, turn, U).astype(np.float64)
        # the sample of index S_r - 1 lies on the spoke's positive side
        ang = np.arctan2(t[:, -1, 1], t[:, -1, 0]) % (2 * np.pi)
        want = (2 * np.pi * np.arange(K) / K + 2 * np.pi * turn / (K * U)) % (2 * np.pi)
        assert np.allclose(ang, want, atol=1e-6)
        # k_m = (m - S_r / 2) / (2 N): from -1/2 (m = 0) to just below +1/2
        r = np.hypot(t[..., 0], t[..., 1])
        assert np.allclose(r[0], np.abs(np.arange(S_r) - S_r / 2) / (2 * N), atol=1e-7)
        assert r.max() <= 0.5 + 1e-7
    with pytest.raises(ValueError):
        synth.radial_trajectory(N, 6, S_r)          # even spoke counts duplicate spokes


def test_scaling_and_noise():
    clean = synth.single_frame(seed=9, N=32, J=8, K=13, sigma=0.0)
    assert np.linalg.norm(clean.y.astype(np.complex128)) == pytest.approx(100.0, rel=1e-6)
    noisy = synth.single_frame(seed=9, N=32, J=8, K=13, sigma=1e-3)
    d = (noisy.y.astype(np.complex128) - clean.y.astype(np.complex128)).ravel()
    # complex Gaussian noise, sigma / sqrt(2) per real component (complex64 storage aside)
    assert np.std(d.real) == pytest.approx(1e-3 / np.sqrt(2), rel=0.05)
    assert np.std(d.imag) == pytest.approx(1e-3 / np.sqrt(2), rel=0.05)
    assert abs(np.mean(d)) < 1e-4
