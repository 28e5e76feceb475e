"""One frame on each of several plans of different grids, coil and spoke
counts as one HIP graph launch (nlinv_reconstruct_multi): every plan's result
equals its own nlinv_reconstruct bit for bit, on the first call (capture), on
replays of the cached graph, for a new argument set, after a member plan's
coil weights change, and for a new plan created after one was destroyed."""
import numpy as np
import pytest

from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(32, 4, 5, 2), (64, 6, 9, 1), (128, 8, 11, 1)]   # (N, J, K, B): grids 64, 128, 256
M, C = 3, 5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()
    return _t


def _plan(torch, i, N, J, K, B):
    """A plan of batch B whose items are the single-frame phantom of seed
    10 i + b on turn b; returns the plan, its gridded data and the turns."""
    from paper_1701_08361_amd import nlinv as nl
    plan = nl.Plan(N, J, K, U=B, batch=B, newton=M, cg=C)
    frames = [synth.single_frame(seed=10 * i + b + 1, N=N, J=J, K=K) for b in range(B)]
    traj = torch.from_numpy(np.stack([f.traj[0] for f in frames])).cuda()
    y = torch.from_numpy(np.stack([f.y[0] for f in frames])).cuda()
    turns = list(range(B))
    z = plan.grid(traj, y, turns=turns)
    return plan, z, turns


def _per_plan(plans, zs, turns, xprevs, inits):
    out = []
    for plan, z, t, xp, ini in zip(plans, zs, turns, xprevs, inits):
        x, img, _ = plan.reconstruct(z, t, xprev=xp, init=ini, want_img=True)
        out.append((x, img))
    return out


def test_multi_reconstruction_equals_per_plan(torch):
    from paper_1701_08361_amd import nlinv as nl
    print(f"[case] multi-plan reconstruction shapes={SHAPES} M={M} C={C}", flush=True)
    built = [_plan(torch, i, *s) for i, s in enumerate(SHAPES)]
    plans = [b[0] for b in built]
    zs = [b[1] for b in built]
    turns = [b[2] for b in built]
    n = len(plans)

    def check(xprevs, inits, what):
        ref = _per_plan(plans, zs, turns, xprevs, inits)
        for rep in range(3):   # capture, then replays of the cached graph
            xs, imgs = nl.reconstruct_multi(plans, zs, turns, xprevs=xprevs, inits=inits, want_img=True)
            torch.cuda.synchronize()
            for i in range(n):
                assert torch.equal(xs[i], ref[i][0]) and torch.equal(imgs[i], ref[i][1]), (what, rep, i)
            # eager work on the same workspaces between the replays
            plans[rep % n].reconstruct(zs[rep % n], turns[rep % n], init=1)
            torch.cuda.synchronize()
        print(f"{what}: every plan equals its own reconstruction (capture and two replays)")
        return ref

    ref = check([None] * n, [1] * n, "unit start")
    # a new argument set: each plan regularised to its previous result
    ref2 = check([r[0] for r in ref], [2] * n, "temporal regularisation")
    assert not torch.equal(ref2[0][0], ref[0][0])
    # a member's coil weights change: the cached graphs of that plan are stale
    gc = plans[1].Gc
    w = torch.full((gc, gc), 0.5, dtype=torch.float32, device="cuda")
    plans[1].set_coil_weights(w)
    ref3 = check([r[0] for r in ref], [2] * n, "changed coil weights")
    assert not torch.equal(ref3[1][0], ref2[1][0])
    plans[1].set_coil_weights(None)
    # a plan destroyed and a new one in its place
    plans[2].close()
    plans[2], zs[2], turns[2] = _plan(torch, 2, *SHAPES[2])
    check([None] * n, [1] * n, "replaced plan")
    for p in plans:
        p.close()


def test_multi_reconstruction_rejects_bad_sets(torch):
    from paper_1701_08361_amd import nlinv as nl
    print("[case] multi-plan reconstruction argument checks", flush=True)
    plan, z, turns = _plan(torch, 0, *SHAPES[0])
    with pytest.raises(nl.NlinvError) as e:     # the same plan twice
        nl.reconstruct_multi([plan, plan], [z, z], [turns, turns])
    assert e.value.code == nl.E_ARG
    plan.timer_enable("toeplitz_rows")         # a kernel timer armed: no capture
    with pytest.raises(nl.NlinvError) as e:
        nl.reconstruct_multi([plan], [z], [turns])
    assert e.value.code == nl.E_STATE
    plan.close()
    st = nl.Plan(32, 4, 5, newton=M, cg=C, static_workspace=True)   # static plans launch eagerly
    zs = torch.zeros(1, 4, 32, 32, dtype=torch.complex64, device="cuda")
    with pytest.raises(nl.NlinvError) as e:
        nl.reconstruct_multi([st], [zs], [[0]])
    assert e.value.code == nl.E_STATE
    st.close()
