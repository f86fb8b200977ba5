"""Host logic of the tile-shape tuner, without a GPU: the timing of one candidate is replaced by
a stub, so these tests check the selection, the bitwise guard and the cache rules only."""
import pytest
import torch

from paper_1001_5341_amd import _native as N
from paper_1001_5341_amd import autotune
from paper_1001_5341_amd import workloads as W

CPU = torch.device("cpu")


@pytest.fixture
def stub(monkeypatch):
    """Candidate timings from a table; waveforms and final-field digests all equal unless a
    candidate is marked (odd: other waveforms; odd_fields: same waveforms, other final fields)."""
    state = {"times": {}, "odd": set(), "odd_fields": set(), "calls": [], "invalid": set()}

    def fake(w, storage, waves, zchunk, steps, device, kernel="fused"):
        key = (waves, zchunk, kernel)
        state["calls"].append(key)
        if key in state["invalid"]:
            raise N.ChfError(-1, "chf_plan_create", "shape not valid for this grid")
        wave = torch.ones(2, 3, 4) + (1.0 if key in state["odd"] else 0.0)
        digest = (1, 2, 3, 4, 5, 6 + (1 if key in state["odd_fields"] else 0))
        return state["times"].get(key, 5.0), (wave, digest), {"vx": 4}

    monkeypatch.setattr(autotune, "_time_candidate", fake)
    monkeypatch.setattr(autotune, "shape_key", lambda w, storage, device=None: f"test/{storage}/{w.nx}x{w.ny}x{w.nz}")
    return state


def test_fastest_candidate_is_cached_and_reused(stub, tmp_path):
    w = W.small_shower()
    path = str(tmp_path / "tune.json")
    cands = [(7, 8, "fused"), (8, 12, "fused_prefetch"), (4, 16, "fused")]
    stub["times"] = {(7, 8, "fused"): 2.0, (8, 12, "fused_prefetch"): 1.5, (4, 16, "fused"): 3.0}
    t = autotune.tune(w, "fp32", cache_path=path, candidates=cands, device=CPU)
    assert (t["waves"], t["z_chunk"], t["kernel"], t["cached"]) == (8, 12, "fused_prefetch", False)
    assert len(stub["calls"]) == 3
    again = autotune.tune(w, "fp32", cache_path=path, candidates=cands, device=CPU)
    assert again["cached"] and (again["waves"], again["z_chunk"], again["kernel"]) == (8, 12, "fused_prefetch")
    assert len(stub["calls"]) == 3
    # a cached shape outside the offered candidates is not used: the shape is tuned again
    again = autotune.tune(w, "fp32", cache_path=path, candidates=[(7, 8, "fused"), (4, 16, "fused")], device=CPU)
    assert not again["cached"] and (again["waves"], again["z_chunk"]) == (7, 8)
    # two-element candidates mean the plain fused sweep
    t = autotune.tune(w, "fp32", cache_path=path, candidates=[(4, 16)], use_cache=False, device=CPU)
    assert t["kernel"] == "fused"


def test_candidate_changing_the_waveforms_is_an_error(stub, tmp_path):
    stub["odd"] = {(8, 12, "fused")}
    with pytest.raises(RuntimeError, match="changes the results"):
        autotune.tune(W.small_shower(), "fp32", cache_path=str(tmp_path / "t.json"),
                      candidates=[(7, 8, "fused"), (8, 12, "fused")], device=CPU)


def test_candidate_changing_only_the_final_fields_is_an_error(stub, tmp_path):
    # the guard compares every node of the final state, not only the observers' waveforms
    stub["odd_fields"] = {(8, 12, "fused")}
    with pytest.raises(RuntimeError, match="changes the results"):
        autotune.tune(W.small_shower(), "fp32", cache_path=str(tmp_path / "t.json"),
                      candidates=[(7, 8, "fused"), (8, 12, "fused")], device=CPU)


def test_field_digest_sees_a_single_changed_value():
    # the digest on CPU tensors: one flipped low mantissa bit anywhere changes it
    class FakePlan:
        def __init__(self, fields):
            self.fields = fields

        def get_field(self, c, stream=None):
            return self.fields[c]

    g = torch.Generator().manual_seed(3)
    base = [torch.rand((5, 7, 9), generator=g) for _ in range(6)]
    d0 = autotune.field_digest(FakePlan(base))
    assert d0 == autotune.field_digest(FakePlan([f.clone() for f in base]))
    for c, idx in [(0, (0, 0, 0)), (3, (4, 6, 8)), (5, (2, 3, 4))]:
        alt = [f.clone() for f in base]
        bits = alt[c].view(torch.int32)
        bits[idx] ^= 1
        d1 = autotune.field_digest(FakePlan(alt))
        assert d1 != d0 and [a != b for a, b in zip(d0, d1)].count(True) == 1


def test_invalid_shapes_are_skipped(stub, tmp_path):
    stub["invalid"] = {(15, 8, "fused")}
    stub["times"] = {(7, 8, "fused"): 2.0}
    t = autotune.tune(W.small_shower(), "fp32", cache_path=str(tmp_path / "t.json"),
                      candidates=[(15, 8, "fused"), (7, 8, "fused")], device=CPU)
    assert (t["waves"], t["z_chunk"]) == (7, 8)
    assert {"waves": 15, "z_chunk": 8, "kernel": "fused", "error": "CHF_EINVAL"} in t["trials"]
    stub["invalid"] = {(15, 8, "fused"), (7, 8, "fused")}
    with pytest.raises(RuntimeError, match="no valid tile shape"):
        autotune.tune(W.small_shower(), "fp32", cache_path=str(tmp_path / "t2.json"),
                      candidates=[(15, 8, "fused"), (7, 8, "fused")], device=CPU)


def test_batch_members_cached_apart_with_a_common_row_count(stub, tmp_path):
    path = str(tmp_path / "tune.json")
    ws = [W.small_shower(seed=1), W.small_shower(seed=2, nz=160), W.small_shower(seed=3, nz=170)]
    cands = [(7, 8, "fused"), (7, 12, "fused"), (8, 8, "fused")]
    stub["times"] = {(8, 8, "fused"): 1.0}
    plan_t = autotune.tune(ws[0], "fp32", cache_path=path, candidates=cands, device=CPU)
    assert (plan_t["waves"], plan_t["z_chunk"]) == (8, 8)
    stub["times"] = {(7, 12, "fused"): 1.0}
    res = autotune.tune_batch(ws, "fp32", cache_path=path, candidates=cands, device=CPU)
    assert [r["waves"] for r in res] == [7, 7, 7] and [r["z_chunk"] for r in res] == [12, 12, 12]
    assert [r["kernel"] for r in res] == ["fused"] * 3
    table = autotune._load(path)
    assert "test/fp32/72x60x150" in table and "test/fp32/72x60x150/batch" in table
    # the plan tuning of the shape is untouched by the batch tuning
    assert (table["test/fp32/72x60x150"]["waves"], table["test/fp32/72x60x150"]["z_chunk"]) == (8, 8)


def test_batch_takes_one_row_count_and_sweep_kind(stub, tmp_path):
    """Members tuned to different shapes share the most common (rows, sweep kind) pair and keep
    their own z chunks."""
    path = str(tmp_path / "tune.json")
    ws = [W.small_shower(seed=1, nz=150), W.small_shower(seed=2, nz=160), W.small_shower(seed=3, nz=170)]
    best = {150: (11, 8, "fused_prefetch"), 160: (11, 16, "fused_prefetch"), 170: (7, 12, "fused")}
    res = []
    for w in ws:
        stub["times"] = {best[w.nz]: 1.0}
        res += autotune.tune_batch([w], "fp32", cache_path=path,
                                   candidates=[(7, 12, "fused"), (11, 8, "fused_prefetch"), (11, 16, "fused_prefetch")],
                                   device=CPU)
    stub["times"] = {}
    res = autotune.tune_batch(ws, "fp32", cache_path=path,
                              candidates=[(7, 12, "fused"), (11, 8, "fused_prefetch"), (11, 16, "fused_prefetch")],
                              device=CPU)
    assert [(r["waves"], r["kernel"]) for r in res] == [(11, "fused_prefetch")] * 3
    assert [r["z_chunk"] for r in res] == [8, 16, 12]
