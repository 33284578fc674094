"""The autotuner: shape buckets, the cache, and (on the GPU) a short tuning
run whose winner is re-checked against the defaults."""
import os

import pytest

from paper_2507_20802_amd import autotune as A


def test_bucket_keys_round_sizes_to_powers_of_two():
    assert A.bucket_key(3, 32768, 33, "MI355X") == "d3_n2^15_r2^5_MI355X"
    assert A.bucket_key(3, 30000, 32, "MI355X") == A.bucket_key(3, 32768, 33, "MI355X")
    assert A.bucket_key(2, 4096, 32, "a b") == "d2_n2^12_r2^5_a_b"
    assert A.bucket_key(2, 4096, 32, "x") != A.bucket_key(3, 4096, 32, "x")


def test_cache_round_trip_and_tuning(tmp_path):
    path = str(tmp_path / "t.json")
    assert A.load_cache(path) == {}
    A.save_cache({"k": {"knobs": {"threads_per_atom": 4, "skin": 0.25, "block_iters": 16}}}, path)
    e = A.load_cache(path)["k"]
    t = A.tuning_of(e["knobs"])
    assert (t.threads_per_atom, t.skin, t.block_iters) == (4, 0.25, 16)
    assert A.tuning_of(A.DEFAULT).threads_per_atom == A.DEFAULT["threads_per_atom"]


def test_every_knob_value_is_tried_once_per_pass():
    seen = [(k, v) for k, vals in A.coordinate_order() for v in vals]
    assert len(seen) == sum(len(v) for v in A.KNOBS.values())
    assert all(v[0] == A.DEFAULT[k] for k, v in A.KNOBS.items())


@pytest.mark.gpu
def test_tuning_run_picks_a_checked_winner(tmp_path):
    path = str(tmp_path / "tune.json")
    entry = A.tune(2, 1000, 4, iters=400, repeats=1, cache=path)
    assert entry["parity"]["ok"]
    for k, v in entry["knobs"].items():
        assert v in A.KNOBS[k]
    assert entry["ms"] <= entry["default_ms"] * 1.0001
    os.environ["AQS_TUNE_CACHE"] = path
    try:
        from paper_2507_20802_amd import Engine
        import aqs_synth as S
        s = S.uniform_glass_start(2, 1000, 3, 11)
        eng = Engine(2, [1000] * 4, s.L, 1e-4, tuning="auto")
        assert eng.tuning.threads_per_atom == entry["knobs"]["threads_per_atom"]
        assert eng.tuning.skin == entry["knobs"]["skin"]
    finally:
        del os.environ["AQS_TUNE_CACHE"]


@pytest.mark.gpu
def test_live_tuning_keeps_the_round(tmp_path):
    """With slots for two chains and their snapshots the tuner also chooses
    graph replay on one replica alone (the critical chain) and times live
    rounds over the critical chain's share of the GPU; the winner makes the
    same decisions and minimisations as the default."""
    path = str(tmp_path / "tune.json")
    entry = A.tune(2, 1000, 5, iters=400, repeats=1, cache=path, live_steps=3, crit_steps=3)
    assert entry["parity"]["ok"] and entry["live"]["same_round_as_default"]
    crit = entry["critical_chain"]["ms_by_use_graph"]
    assert set(crit) == {"0", "1"}
    assert crit[str(entry["knobs"]["use_graph"])] == min(crit.values())
    for k, v in entry["knobs"].items():
        assert v in (A.KNOBS.get(k) or A.LIVE_KNOBS[k])
    assert set(A.LIVE_KNOBS) <= set(entry["knobs"])
    assert entry["live"]["ms"] <= entry["live"]["default_ms"] * 1.0001


def test_graph_replay_is_chosen_on_the_critical_chain(tmp_path, monkeypatch):
    """Host logic of the tuner with stubbed timings: for a shape that holds
    live rounds, graph replay is decided by one replica's chain (the
    critical chain), not by the batch, and the batch's winner is kept for
    every other knob; a shape without live rounds keeps the batch's choice."""
    def trial(dim, n, n_rep, s, is_pos, knobs, iters, dg, steps=3):
        if n_rep == 1:                       # one replica: replay pays
            return 1.0 if knobs["use_graph"] else 1.2
        t = 2.0 - (0.1 if knobs["skin"] == 0.25 else 0.0)
        return t + (0.01 if knobs["use_graph"] else 0.0)   # the batch: replay costs a little

    monkeypatch.setattr(A, "_glass", lambda dim, n, seed: (None, None))
    monkeypatch.setattr(A, "_trial", trial)
    monkeypatch.setattr(A, "_same_inherent_structure",
                        lambda *a, **k: {"ok": True, "energy_rel": 0.0, "max_disp": 0.0})
    monkeypatch.setattr(A, "_live_trial", lambda dim, n, n_rep, s, is_pos, knobs, dg, steps:
                        (1.0 + 0.1 * knobs["live_xcds"], ([], [])))
    monkeypatch.setattr(A, "_same_round", lambda a, b: True)
    monkeypatch.setattr(A, "device_name", lambda: "stub")
    path = str(tmp_path / "t.json")
    live = A.tune(3, 1000, 5, repeats=1, cache=path)
    assert live["knobs"]["use_graph"] == 1 and live["knobs"]["skin"] == 0.25
    assert live["critical_chain"]["ms_by_use_graph"] == {"0": 1200.0, "1": 1000.0}
    assert live["knobs"]["live_xcds"] == 0
    batch = A.tune(3, 1000, 4, repeats=1, cache=path)
    assert batch["knobs"]["use_graph"] == 0 and "critical_chain" not in batch
    assert set(A.load_cache(path)) == {A.bucket_key(3, 1000, 5, "stub"), A.bucket_key(3, 1000, 4, "stub")}
