"""Pins of the oracle's frame-series schedules (Sec. 3.3, temporal
decomposition, equation for h(n, m)).

The schedule is checked against the properties the equation fixes: frames up
to l follow strictly; later frames take a source in [n-o, n-1]; the members
of a group never depend on each other before the last Newton step.  The
reconstruction is checked against the special cases that reduce to the strict
order: o = 1, a single Newton step (M = 1, where h(n, M-1) = n-1 is the only
step), and the first frame of every group (whose source is n-1).
"""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth


@pytest.mark.parametrize("F", [0, 1, 2, 7, 15, 31])
@pytest.mark.parametrize("l", [0, 1, 3, 5])
@pytest.mark.parametrize("o", [1, 2, 3, 5])
def test_relaxed_schedule_properties(F, l, o):
    src = O.relaxed_sources(F, l, o)
    assert len(src) == F
    for n, s in enumerate(src):
        if n == 0:
            assert s == -1
        elif n <= l:
            assert s == n - 1                      # strict order up to l
        else:
            assert n - o <= s <= n - 1             # source within [n-o, n-1]
    # groups: frames after l sharing a source are consecutive, at most o long,
    # and start right after their source (the most recent frame that can be done)
    groups = {}
    for n in range(l + 1, F):
        groups.setdefault(src[n], []).append(n)
    for s, members in groups.items():
        assert members == list(range(members[0], members[0] + len(members)))
        assert len(members) <= o
        assert s == members[0] - 1
    # every group but the last is full
    sizes = [len(m) for _, m in sorted(groups.items())]
    assert all(k == o for k in sizes[:-1])


def test_relaxed_schedule_o1_and_large_l_are_strict():
    for F, l in [(10, 0), (10, 4), (6, 9)]:
        assert O.relaxed_sources(F, l, 1) == [n - 1 for n in range(F)]
    assert O.relaxed_sources(8, 7, 4) == [n - 1 for n in range(8)]
    with pytest.raises(ValueError):
        O.relaxed_sources(4, 0, 0)


def _tiny_series(frames=6, N=8, J=2, K=5, U=3, seed=11):
    ser = synth.real_time_series(seed=seed, N=N, J=J, J_phys=3, K=K, U=U, frames=frames)
    g = O.Geometry.make(N, J)
    zs = [O.grid(ser.y[f].astype(np.complex128), ser.traj[f].astype(np.float64), g.R) for f in range(frames)]
    Ps = [O.psf_kernel(ser.traj[f].astype(np.float64), g.R, g.G) for f in range(frames)]
    return g, zs, Ps


def test_series_o1_equals_strict_chain():
    """o = 1 is the strict order: each frame starts from, and is regularised
    towards, the previous result (bit-identical arithmetic)."""
    g, zs, Ps = _tiny_series()
    strict = O.reconstruct_series(g, zs, Ps, None, newton=3, cg_iters=4)
    relaxed = O.reconstruct_series(g, zs, Ps, O.relaxed_sources(len(zs), 1, 1), newton=3, cg_iters=4)
    chain, prev = [], None
    for z, P in zip(zs, Ps):
        prev = O.reconstruct(g, z, P, xprev=prev, x0=prev, newton=3, cg_iters=4)
        chain.append(prev)
    for a, b, c in zip(strict, relaxed, chain):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_series_single_newton_step_is_strict():
    """M = 1: the only step is m = M-1, for which h(n, m) = n-1, so any l, o
    give the strict result."""
    g, zs, Ps = _tiny_series()
    strict = O.reconstruct_series(g, zs, Ps, None, newton=1, cg_iters=5)
    relaxed = O.reconstruct_series(g, zs, Ps, O.relaxed_sources(len(zs), 0, 3), newton=1, cg_iters=5)
    for a, b in zip(strict, relaxed):
        assert np.array_equal(a, b)


def test_series_group_structure():
    """The first frame of each group continues strictly from its predecessor;
    later members differ from the strict continuation (their first M-1 steps
    use an older frame), and the last step uses x_{n-1}."""
    g, zs, Ps = _tiny_series(frames=7)
    M, C = 3, 4
    src = O.relaxed_sources(len(zs), 1, 3)          # groups {2, 3, 4}, {5, 6}
    assert src == [-1, 0, 1, 1, 1, 4, 4]
    out = O.reconstruct_series(g, zs, Ps, src, newton=M, cg_iters=C)
    for n in (2, 5):                                # group heads: strict continuation
        ref = O.reconstruct(g, zs[n], Ps[n], xprev=out[n - 1], x0=out[n - 1], newton=M, cg_iters=C)
        assert np.array_equal(out[n], ref)
    for n in (3, 4, 6):                             # members: M-1 steps from the source, then one step
        x = O.reconstruct(g, zs[n], Ps[n], xprev=out[src[n]], x0=out[src[n]], newton=M - 1, cg_iters=C)
        ref = x + O.newton_step(g, x, out[n - 1], zs[n], Ps[n], O.alpha_schedule(M)[M - 1], C)
        assert np.array_equal(out[n], ref)
        strict = O.reconstruct(g, zs[n], Ps[n], xprev=out[n - 1], x0=out[n - 1], newton=M, cg_iters=C)
        assert not np.array_equal(out[n], strict)
