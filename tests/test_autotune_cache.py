"""The batch autotuner's result cache, on the CPU (the timed runs are replaced
by a stand-in, so no GPU call is made)."""
import json

import numpy as np

from paper_2607_07816_amd import batch as B
from paper_2607_07816_amd import circuits as C


def _items(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(6, 12))
        c = C.peaked_circuit(n, 2, 0.01, seed * 100 + i)
        out.append((c, 1 << int(rng.integers(4, 8)), 0.0))
    return out


def test_cache_hit_skips_the_timed_runs(tmp_path, monkeypatch):
    calls = []

    def fake_run(sub, precision, streams, graph_steps, packed=None, sort=(0, "8x16")):
        calls.append((streams, graph_steps, sort))
        return [], 1.0 / streams + 0.1 * (graph_steps > 0)

    monkeypatch.setattr(B, "run_batch", fake_run)
    monkeypatch.setattr(B, "pack", lambda sub: None)
    items = _items(1, 12)
    cache = str(tmp_path / "tune.json")
    cands = [(4, 0), (8, 0), (8, 16)]
    sorts = [(0, "8x16")]
    choice, t1 = B.autotune(items, "c64", candidates=cands, cache=cache, sorts=sorts)
    assert choice == (8, 0, 0, "8x16") and len(calls) == 3
    assert set(t1) == {c + (0, "8x16") for c in cands}
    data = json.load(open(cache))
    assert len(data) == 1
    # same batch: served from the file
    choice2, t2 = B.autotune(items, "c64", candidates=cands, cache=cache, sorts=sorts)
    assert choice2 == choice and t2 == t1 and len(calls) == 3
    # another precision, another candidate list or another mix: tuned again
    B.autotune(items, "c128", candidates=cands, cache=cache, sorts=sorts)
    B.autotune(items, "c64", candidates=cands[:2], cache=cache, sorts=sorts)
    B.autotune(_items(2, 9), "c64", candidates=cands, cache=cache, sorts=sorts)
    assert len(calls) == 3 + 3 + 2 + 3
    assert len(json.load(open(cache))) == 4


def test_sort_policies_timed_at_the_best_stream_setting(tmp_path, monkeypatch):
    calls = []
    cost = {(0, "8x16"): 1.0, (20, "11x16"): 0.7, (20, "8x8"): 0.9}

    def fake_run(sub, precision, streams, graph_steps, packed=None, sort=(0, "8x16")):
        calls.append((streams, graph_steps, sort))
        return [], cost[sort] / streams

    monkeypatch.setattr(B, "run_batch", fake_run)
    monkeypatch.setattr(B, "pack", lambda sub: None)
    cache = str(tmp_path / "tune.json")
    sorts = list(cost)
    choice, t = B.autotune(_items(5, 8), "c64", candidates=[(2, 0), (4, 0)], cache=cache, sorts=sorts)
    # streams first at the first sort policy, then the others at 4 streams
    assert calls == [(2, 0, (0, "8x16")), (4, 0, (0, "8x16")), (4, 0, (20, "11x16")), (4, 0, (20, "8x8"))]
    assert choice == (4, 0, 20, "11x16")
    # another sort list is another key
    B.autotune(_items(5, 8), "c64", candidates=[(2, 0), (4, 0)], cache=cache, sorts=sorts[:2])
    assert len(calls) == 7
    choice2, _ = B.autotune(_items(5, 8), "c64", candidates=[(2, 0), (4, 0)], cache=cache, sorts=sorts)
    assert choice2 == choice and len(calls) == 7


def test_signature_depends_on_shape_only():
    a = _items(3, 8)
    assert B.batch_signature(a) == B.batch_signature(list(reversed(a)))
    assert B.batch_signature(a) != B.batch_signature(a[:-1])
    assert B.batch_signature(a, "c64") != B.batch_signature(a, "c128")


def test_unreadable_cache_is_ignored(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "run_batch", lambda sub, prec, s, g, packed=None, sort=None: ([], float(s)))
    monkeypatch.setattr(B, "pack", lambda sub: None)
    cache = tmp_path / "tune.json"
    cache.write_text("not json")
    choice, _ = B.autotune(_items(4, 4), "c64", candidates=[(2, 0), (1, 0)], cache=str(cache))
    assert choice[:2] == (1, 0)
    assert len(json.load(open(cache))) == 1
