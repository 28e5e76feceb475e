"""The streaming server (paper_1701_08361_amd.serve): per-slice pipelines on
their own streams give exactly the results of the direct C-ABI calls, and
admission respects the device-memory budget."""
import numpy as np
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


def test_server_matches_direct_calls(torch):
    from paper_1701_08361_amd import nlinv, serve
    N, J, Jp, K, U, M, C, F = 32, 4, 8, 5, 2, 3, 4, 4
    print(f"[case] server N={N} J={J} Jp={Jp} K={K} U={U} M={M} C={C} frames={F}", flush=True)
    shapes = [(N, J, Jp, K), (64, 6, 12, 7)]
    sers = [synth.real_time_series(seed=91 + q, N=n, J=j, J_phys=jp, K=k, U=U, frames=F, compress=False)
            for q, (n, j, jp, k) in enumerate(shapes)]
    for shared in (False, True):
        srv = serve.Server(budget_bytes=4 << 30, shared_streams=shared)
        outs = {}
        for (n, j, jp, k), ser in zip(shapes, sers):
            tr = torch.from_numpy(ser.traj).cuda()
            srv.admit(f"s{n}", n, j, jp, k, U, tr[:U], torch.from_numpy(ser.y[0]).cuda(), newton=M, cg=C)
        host = [torch.from_numpy(ser.y).pin_memory() for ser in sers]
        for f in range(F):
            for (n, j, jp, k), ser, h in zip(shapes, sers, host):
                ev, img = srv.submit(f"s{n}", h[f], torch.from_numpy(ser.traj[f]).cuda(), int(ser.turn[f]))
                outs[(n, f)] = (ev, img)
            srv.synchronize()
            for (n, *_), _s in zip(shapes, sers):
                outs[(n, f)] = outs[(n, f)][1].clone()
        # the same steps through the plan directly
        for (n, j, jp, k), ser in zip(shapes, sers):
            plan = nlinv.Plan(n, j, k, U=U, newton=M, cg=C, cg_passes=4)    # the server's form
            tr = torch.from_numpy(ser.traj).cuda()
            for t in range(U):
                plan.psf(tr[t].contiguous(), t)
            cc = plan.compression_matrix(torch.from_numpy(ser.y[0]).cuda())
            prev = None
            for f in range(F):
                y = plan.compress(cc, torch.from_numpy(ser.y[f:f + 1]).cuda())
                z = plan.grid(tr[f:f + 1], y, turns=[int(ser.turn[f])])
                x, img, _ = plan.reconstruct(z, [int(ser.turn[f])], xprev=prev, init=1 if f == 0 else 2,
                                             want_img=True)
                prev = x
                assert torch.equal(img[0].cpu(), outs[(n, f)]), (shared, n, f)
            plan.close()
        for (n, *_) in shapes:
            srv.release(f"s{n}")
        assert srv.used == 0


def test_server_admission_budget(torch):
    from paper_1701_08361_amd import serve
    N, J, Jp, K, U = 32, 4, 8, 5, 1
    ser = synth.real_time_series(seed=95, N=N, J=J, J_phys=Jp, K=K, U=U, frames=1, compress=False)
    need = serve.Server.slice_bytes(N, J, Jp, K, U, 7, 20)
    srv = serve.Server(budget_bytes=2 * need - 1)
    tr = torch.from_numpy(ser.traj).cuda()
    calib = torch.from_numpy(ser.y[0]).cuda()
    srv.admit("a", N, J, Jp, K, U, tr, calib)
    with pytest.raises(serve.BudgetError):
        srv.admit("b", N, J, Jp, K, U, tr, calib)
    assert list(srv.slices) == ["a"] and srv.used == need
    srv.release("a")
    srv.admit("b", N, J, Jp, K, U, tr, calib)
    assert srv.used == need


def test_library_budget_admission(torch):
    """nlinv_set_budget: plan creation beyond the device's workspace budget
    fails with NLINV_E_BUDGET; destroying a plan returns its share."""
    import gc
    from paper_1701_08361_amd import nlinv
    print("[case] library budget admission", flush=True)
    gc.collect()
    dev = torch.cuda.current_device()
    need = nlinv.workspace_size(nlinv.make_params(32, 4, 5))
    base = nlinv.budget_used(dev)
    nlinv.set_budget(dev, base + 2 * need)
    try:
        a = nlinv.Plan(32, 4, 5)
        b = nlinv.Plan(32, 4, 5)
        assert nlinv.budget_used(dev) == base + 2 * need
        with pytest.raises(nlinv.NlinvError) as ei:
            nlinv.Plan(32, 4, 5)
        assert ei.value.code == nlinv.E_BUDGET
        a.close()
        assert nlinv.budget_used(dev) == base + need
        c = nlinv.Plan(32, 4, 5)
        c.close()
        b.close()
        assert nlinv.budget_used(dev) == base
    finally:
        nlinv.set_budget(dev, 0)
