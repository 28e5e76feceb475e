"""The autotuning database and its selection rules (Sec. 3.3, autotuning),
with a stand-in for the measured run (no GPU)."""
import json

import pytest

from paper_1701_08361_amd import autotune as AT


def proto(**kw):
    p = dict(mode="single-slice", N=160, J=10, K=15, U=5, frames=50, newton=7, cg=20)
    p.update(kw)
    return p


def fake_rate(c):
    # a made-up rate with one best setting: T = 3 with graphs
    return 10.0 + 5.0 * c["graphs"] - abs(c["T"] - 3) * 1.5


def test_search_space_matches_the_papers_limits():
    """One GPU: T = 1..8 with A = 1, each with graphs off and on.  Eight GPUs:
    the paper's 16 (T, A) pairs (A = 1: T <= 8, A = 2: T <= 4, A = 3, 4: T <= 2)."""
    one = AT.search_space(1)
    assert len(one) == 16 and {c["A"] for c in one} == {1}
    assert sorted({c["T"] for c in one}) == list(range(1, 9))
    eight = {(c["T"], c["A"]) for c in AT.search_space(8)}
    paper = {(t, 1) for t in range(1, 9)} | {(t, 2) for t in range(1, 5)} | {(t, a) for t in (1, 2) for a in (3, 4)}
    assert eight == paper and len(paper) == 16


def test_tile_schedule_dimension():
    """With tiles, every (T, A, graphs) setting comes with each column-pass
    tile schedule; the learning mode then measures the schedules too."""
    sp = AT.search_space(1, tiles=(8, 4))
    assert len(sp) == 32 and {c["col_tile"] for c in sp} == {4, 8}
    assert {(c["T"], c["graphs"]) for c in sp} == {(c["T"], c["graphs"]) for c in AT.search_space(1)}
    with pytest.raises(ValueError):
        AT.search_space(1, tiles=(16,))
    rate = lambda c: fake_rate(c) + (0.5 if c["col_tile"] == 4 else 0.0)
    tuner = AT.Autotuner(AT.TuningDB(), learning=True, tiles=(8, 4))
    best = tuner.learn(proto(), rate)
    assert best == {"T": 3, "A": 1, "graphs": True, "col_tile": 4}


def test_learning_mode_tries_every_setting_then_the_best_wins(tmp_path):
    db = AT.TuningDB(str(tmp_path / "tune.json"))
    tuner = AT.Autotuner(db, learning=True)
    p = proto()
    seen = []
    while tuner.untried(p):
        c = tuner.choose(p)
        assert c not in seen            # never a setting that is already recorded
        seen.append(c)
        tuner.record(p, c, fake_rate(c))
    assert len(seen) == 16
    assert tuner.choose(p) == {"T": 3, "A": 1, "graphs": True}    # nothing left to learn: the best
    assert AT.Autotuner(db).choose(p) == {"T": 3, "A": 1, "graphs": True}


def test_learn_helper_and_persistence(tmp_path):
    path = str(tmp_path / "tune.json")
    best = AT.Autotuner(AT.TuningDB(path), learning=True).learn(proto(), fake_rate)
    assert best == {"T": 3, "A": 1, "graphs": True}
    again = AT.TuningDB(path)
    assert len(again.records) == 16
    assert again.lookup(proto())[0] == ({"T": 3, "A": 1, "graphs": True}, fake_rate(best))
    assert json.load(open(path))[0]["protocol"] == proto()


def test_unseen_protocol_takes_the_nearest_recorded_one():
    db = AT.TuningDB()
    db.insert(proto(frames=25), {"T": 2, "A": 1, "graphs": True}, 50.0)
    db.insert(proto(frames=25), {"T": 1, "A": 1, "graphs": True}, 40.0)
    db.insert(proto(frames=200), {"T": 5, "A": 1, "graphs": True}, 90.0)
    db.insert(proto(frames=30, mode="phase-contrast"), {"T": 8, "A": 1, "graphs": False}, 99.0)
    tuner = AT.Autotuner(db)
    assert tuner.choose(proto(frames=30)) == {"T": 2, "A": 1, "graphs": True}
    assert tuner.choose(proto(frames=150)) == {"T": 5, "A": 1, "graphs": True}
    # another imaging mode is never "near": only its own records count
    assert tuner.choose(proto(frames=30, mode="dual-slice")) == {"T": 1, "A": 1, "graphs": True}
    assert tuner.choose(proto(frames=30, mode="phase-contrast")) == {"T": 8, "A": 1, "graphs": False}


def test_database_rejects_bad_records(tmp_path):
    db = AT.TuningDB()
    with pytest.raises(ValueError):
        db.insert(proto(), {"T": 1, "A": 1, "graphs": True}, 0.0)
    with pytest.raises(ValueError):
        db.insert({"N": 160}, {"T": 1, "A": 1, "graphs": True}, 1.0)
    bad = tmp_path / "bad.json"
    bad.write_text('{"not": "a list"}')
    with pytest.raises(ValueError):
        AT.TuningDB(str(bad))


def test_search_space_with_pass_fusion():
    """With passes, every setting comes with each CG pass fusion; a faster
    four-pass form is found and recorded."""
    sp = AT.search_space(1, tiles=(8, 4), passes=(6, 4))
    assert len(sp) == 64 and {c["cg_passes"] for c in sp} == {4, 6}
    assert len({tuple(sorted(c.items())) for c in sp}) == 64
    with pytest.raises(ValueError):
        AT.search_space(1, passes=(5,))
    rate = lambda c: fake_rate(c) + (0.25 if c["cg_passes"] == 4 else 0.0) + (0.5 if c["col_tile"] == 4 else 0.0)
    tuner = AT.Autotuner(AT.TuningDB(), learning=True, tiles=(8, 4), passes=(6, 4))
    best = tuner.learn(proto(), rate)
    assert best == {"T": 3, "A": 1, "graphs": True, "col_tile": 4, "cg_passes": 4}


def test_search_space_with_factorisation():
    sp = AT.search_space(1, passes=(6, 4), splits=(0, 1))
    assert len(sp) == 64 and {c["fft_split"] for c in sp} == {0, 1}
    with pytest.raises(ValueError):
        AT.search_space(1, splits=(2,))
    rate = lambda c: fake_rate(c) + (0.3 if c["fft_split"] == 1 else 0.0)
    tuner = AT.Autotuner(AT.TuningDB(), learning=True, splits=(0, 1))
    assert tuner.learn(proto(), rate) == {"T": 3, "A": 1, "graphs": True, "fft_split": 1}
