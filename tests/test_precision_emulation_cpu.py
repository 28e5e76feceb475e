"""The pass-structure emulator behind the precision choices (float64
intermediates in every Newton step): with no rounding point it reproduces the
oracle's IRGNM, and rounding the half-transformed grid to complex64 in every
operator application moves the result several times more than the library's
complex64 storage of the coil images, unknowns and channel products.  The
160 px figures (where the float32 grid misses 1e-3) come from running
tests/precision_emulation.py as a script (a few minutes)."""
import numpy as np

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth
from precision_emulation import errors, reconstruct


def _case():
    s = synth.single_frame(seed=1, N=64, J=8, K=13)
    g = O.Geometry.make(64, 8)
    z = O.grid(s.y[0], s.traj[0], g.R)
    P = O.psf_kernel(s.traj[0], g.R, g.G)
    return g, z, P


def test_emulator_without_rounding_is_the_oracle():
    g, z, P = _case()
    ref = O.reconstruct(g, z, P, newton=7, cg_iters=10)
    x = reconstruct(g, z, P, (), newton=7, cg_iters=10)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-9


def test_float32_grid_moves_the_result_more_than_the_library_storage():
    g, z, P = _case()
    ref = O.reconstruct(g, z, P, newton=7, cg_iters=10)
    lib = errors(g, reconstruct(g, z, P, {"co", "x", "pr"}, newton=7, cg_iters=10), ref)
    grid32 = errors(g, reconstruct(g, z, P, {"co", "x", "pr", "u2"}, newton=7, cg_iters=10), ref)
    print(f"64 px: library storage {lib[0]:.1e}, + float32 grid {grid32[0]:.1e}")
    assert lib[0] < 1e-5 and grid32[0] > 2 * lib[0]
