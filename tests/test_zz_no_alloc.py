"""Plans on the library's static workspace (nlinv_plan_create_static, for
callers that cannot allocate device memory) against plans on a caller
workspace (nlinv_plan_create): the same gridding and reconstruction, bit for
bit, on two plans in a row, the second of a smaller problem, so that nothing
depends on what the previous plan left in the shared array."""
import gc

import pytest

from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()            # fails loudly when the HIP library is missing
    return _t


def _frame(torch, N, J, K, M, C, seed, static):
    from paper_1701_08361_amd import nlinv
    s = synth.single_frame(seed=seed, N=N, J=J, K=K)
    plan = nlinv.Plan(N, J, K, newton=M, cg=C, static_workspace=static)
    try:
        traj = torch.from_numpy(s.traj).cuda()
        y = torch.from_numpy(s.y).cuda()
        z = plan.grid(traj, y, turns=[0])
        ze = plan.grid(traj, y)                       # exact sum (split partial sums in the workspace)
        x, img, coils = plan.reconstruct(z, [0], want_img=True, want_coils=True)
        plan.sync()
        return [t.clone() for t in (z, ze, x, img, coils)]
    finally:
        plan.close()


@pytest.mark.parametrize("N,J,K,M,C,seed", [(160, 10, 15, 3, 6, 2), (64, 8, 13, 7, 10, 1)])
def test_static_plan_equals_workspace_plan(torch, N, J, K, M, C, seed):
    print(f"[case] static workspace N={N} J={J} K={K} M={M} C={C}", flush=True)
    ref = _frame(torch, N, J, K, M, C, seed, False)
    got = _frame(torch, N, J, K, M, C, seed, True)
    for name, a, b in zip(("z", "z exact", "x", "img", "coils"), ref, got):
        assert torch.equal(a, b), name


def test_one_static_plan_per_device(torch):
    from paper_1701_08361_amd import nlinv
    print("[case] static workspace: one live plan per device", flush=True)
    gc.collect()
    a = nlinv.Plan(32, 3, 5, static_workspace=True)
    try:
        with pytest.raises(nlinv.NlinvError) as ei:
            nlinv.Plan(32, 3, 5, static_workspace=True)
        assert ei.value.code == nlinv.E_STATE
        with pytest.raises(nlinv.NlinvError) as ei:
            a.set_graphs(True)
        assert ei.value.code == nlinv.E_STATE
    finally:
        a.close()
    b = nlinv.Plan(32, 3, 5, static_workspace=True)      # free again after destroy
    b.close()
