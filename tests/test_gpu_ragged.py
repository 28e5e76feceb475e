"""The CG operator of plans of three grid sides with one ragged Toeplitz row
pass (nlinv_apply_normal_multi: one persistent launch over the tiles of every
shape, each shape on its own grid): the same result as nlinv_apply_normal per plan,
bit for bit, and the oracle's operator at the operator bar."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(128, 8, 11, 2), (160, 10, 15, 1), (192, 16, 21, 2)]   # (N, J, K, B): grids 256, 320, 384


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()
    return _t


def _plans(torch, shapes):
    from paper_1701_08361_amd import nlinv as nl
    out = []
    for i, (N, J, K, B) in enumerate(shapes):
        plan = nl.Plan(N, J, K, U=B, batch=B)
        trajs = [synth.radial_trajectory(N, K, 2 * N, b, B) for b in range(B)]
        for b in range(B):
            plan.psf(torch.from_numpy(trajs[b]).cuda(), b)
        g = O.Geometry.make(N, J)
        x = np.stack([synth.random_xhat(100 + 10 * i + b, g.R, J, g.Gc, 1.0, 0.3) for b in range(B)])
        p = np.stack([synth.random_xhat(200 + 10 * i + b, g.R, J, g.Gc, 1.0, 0.3) for b in range(B)])
        out.append((plan, g, trajs, x, p, 0.1 * (i + 1)))
    return out


@pytest.mark.parametrize("which", [(0, 1, 2), (2, 0), (1,)])
def test_ragged_operator_equals_per_plan(torch, which):
    from paper_1701_08361_amd import nlinv as nl
    shapes = [SHAPES[i] for i in which]
    print(f"[case] ragged operator shapes={shapes}", flush=True)
    ps = _plans(torch, shapes)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    turns = [list(range(B)) for (_, _, _, B) in shapes]
    xs, pv = [cu(t[3]) for t in ps], [cu(t[4]) for t in ps]
    qm = nl.apply_normal_multi([t[0] for t in ps], turns, xs, [t[5] for t in ps], pv)
    for (plan, g, trajs, x, p, a), tr, xd, pd, q in zip(ps, turns, xs, pv, qm):
        q1 = plan.apply_normal(tr, xd, pd, a)
        torch.cuda.synchronize()
        assert torch.equal(q, q1)
        P = O.psf_kernel(trajs[0], g.R, g.G)
        ref = O.normal(g, x[0].astype(np.complex128), p[0].astype(np.complex128), P) + a * p[0]
        got = q.cpu().numpy()[0].astype(np.complex128)
        e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"G={g.G}: equal to the per-plan operator; item 0 vs oracle rel {e:.2e}")
        assert e < 1e-4
    for t in ps:
        t[0].close()


def test_ragged_operator_rejects_bad_sets(torch):
    from paper_1701_08361_amd import nlinv as nl
    print("[case] ragged operator argument checks", flush=True)
    small = nl.Plan(32, 2, 5)
    a = _plans(torch, [SHAPES[1]])[0]
    b = _plans(torch, [SHAPES[1]])[0]
    cu = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    g = O.Geometry.make(32, 2)
    xs = cu(synth.random_xhat(1, g.R, 2, g.Gc)[None])
    with pytest.raises(nl.NlinvError) as e:     # grid 64 is not one of the ragged pass's sides
        nl.apply_normal_multi([small], [[0]], [xs], [0.0], [xs.clone()])
    assert e.value.code == nl.E_SIZE
    with pytest.raises(nl.NlinvError) as e:     # two plans of one grid side
        nl.apply_normal_multi([a[0], b[0]], [[0], [0]], [cu(a[3]), cu(b[3])], [0.0, 0.0], [cu(a[4]), cu(b[4])])
    assert e.value.code == nl.E_ARG
    for p in (small, a[0], b[0]):
        p.close()
