"""The autotuner's runner on the GPU: whole series through the C-ABI under
each setting (Sec. 3.3, autotuning)."""
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


def test_runner_settings_and_learning(torch, tmp_path):
    from paper_1701_08361_amd import autotune as AT
    from paper_1701_08361_amd import nlinv
    N, J, K, U, M, C, F = 32, 4, 5, 2, 3, 4, 9
    print(f"[case] autotune runner N={N} J={J} K={K} U={U} M={M} C={C} frames={F}", flush=True)
    ser = synth.real_time_series(seed=81, N=N, J=J, J_phys=6, K=K, U=U, frames=F)
    traj = torch.from_numpy(ser.traj).cuda()
    y = torch.from_numpy(ser.y).cuda()
    turns = [int(t) for t in ser.turn]
    run = lambda c: AT.run_series(nlinv, torch, traj, y, turns, c, M, C, U)
    # graphs change the launch path, never the result
    for T in (1, 3):
        fa, ia = run({"T": T, "A": 1, "graphs": False})
        fb, ib = run({"T": T, "A": 1, "graphs": True})
        assert fa > 0 and fb > 0
        assert torch.equal(ia, ib), T
    # the column-pass tile schedule changes the decomposition, never the result
    _, i4 = run({"T": 3, "A": 1, "graphs": True, "col_tile": 4})
    assert torch.equal(i4, ib)
    # the strict setting reproduces plain frame-by-frame reconstruction
    plan = nlinv.Plan(N, J, K, U=U, newton=M, cg=C)
    for t in range(U):
        plan.psf(traj[t].contiguous(), t)
    prev = None
    for f in range(F):
        z = plan.grid(traj[f:f + 1], y[f:f + 1], turns=[turns[f]])
        x, img, _ = plan.reconstruct(z, [turns[f]], xprev=prev, init=1 if f == 0 else 2, want_img=True)
        prev = x
    _, i1 = run({"T": 1, "A": 1, "graphs": True})
    assert torch.equal(i1, img[0])
    # both settings against the oracle's schedules (strict; groups of 3 after
    # l = U strict frames, the equation for h(n, m))
    _, i3 = run({"T": 3, "A": 1, "graphs": True})
    g = O.Geometry.make(N, J)
    zs = [O.grid(ser.y[f], ser.traj[f], g.R) for f in range(F)]
    Ps = [O.psf_kernel(ser.traj[f], g.R, g.G) for f in range(F)]
    strict = O.reconstruct_series(g, zs, Ps, None, newton=M, cg_iters=C)
    relaxed = O.reconstruct_series(g, zs, Ps, O.relaxed_sources(F, U, 3), newton=M, cg_iters=C)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    e1 = rel(i1.cpu().numpy(), O.image(g, strict[-1]))
    e3 = rel(i3.cpu().numpy(), O.image(g, relaxed[-1]))
    d = rel(O.image(g, relaxed[-1]), O.image(g, strict[-1]))
    # the four-pass CG iteration changes the rounding, not the method
    _, i34 = run({"T": 3, "A": 1, "graphs": False, "cg_passes": 4})
    e34 = rel(i34.cpu().numpy(), O.image(g, relaxed[-1]))
    print(f"last frame vs oracle: T=1 {e1:.2e}, T=3 {e3:.2e}, T=3 four-pass {e34:.2e} "
          f"(relaxed vs strict {d:.2e})")
    assert e1 < 1e-3 and e3 < 1e-3 and e34 < 1e-3 and d > 10 * e3
    # learning over a reduced space records every setting; the choice is the fastest
    db = AT.TuningDB(str(tmp_path / "tune.json"))
    tuner = AT.Autotuner(db, max_T=2, learning=True)
    p = dict(mode="single-slice", N=N, J=J, K=K, U=U, frames=F, newton=M, cg=C)
    best = tuner.learn(p, lambda c: run(c)[0])
    assert len(db.records) == 4 and best == db.lookup(p)[0][0]
    assert AT.Autotuner(AT.TuningDB(str(tmp_path / "tune.json"))).choose(p) == best
    with pytest.raises(ValueError):
        run({"T": 1, "A": 2, "graphs": True})
