"""Pins of the oracle's channel compression (Sec. 3.1, preprocessing)."""
import numpy as np

from oracle import nlinv_oracle as O


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_compression_recovers_a_rank_J_subspace():
    """Data confined to a J-dimensional channel subspace: the compression's
    projector is that subspace's projector and no energy is lost."""
    rng = np.random.default_rng(1)
    Jp, J, S = 12, 4, 300
    A, _ = np.linalg.qr(crand(rng, Jp, J))              # orthonormal basis of the subspace
    y0 = A @ crand(rng, J, S)
    cc = O.compression_matrix(y0, J)
    assert np.allclose(cc @ cc.conj().T, np.eye(J), atol=1e-12)
    assert np.allclose(cc.conj().T @ cc, A @ A.conj().T, atol=1e-10)
    assert abs(np.linalg.norm(O.compress(cc, y0)) - np.linalg.norm(y0)) < 1e-10 * np.linalg.norm(y0)


def test_compression_keeps_the_largest_channel_energies():
    """Independent channels of distinct power: the compression keeps exactly
    the J strongest ones (up to a phase per row)."""
    rng = np.random.default_rng(2)
    powers = np.array([1.0, 9.0, 0.25, 4.0, 16.0, 0.5])
    y0 = np.diag(np.sqrt(powers)) @ np.eye(6, 6)        # orthogonal channel signals
    cc = O.compression_matrix(y0, 3)
    keep = np.argsort(powers)[::-1][:3]
    for row, k in zip(cc, keep):
        assert abs(abs(row[k]) - 1.0) < 1e-12
        assert np.allclose(np.delete(row, k), 0.0, atol=1e-12)


def test_compress_is_the_channel_sum():
    rng = np.random.default_rng(3)
    cc, y = crand(rng, 3, 5), crand(rng, 2, 5, 7)
    ref = np.zeros((2, 3, 7), complex)
    for b in range(2):
        for j in range(3):
            for s in range(7):
                ref[b, j, s] = sum(cc[j, p] * y[b, p, s] for p in range(5))
    assert np.allclose(O.compress(cc, y), ref, atol=1e-13)
