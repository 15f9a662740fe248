"""Batches of circuits (sts_batch_run) against the same circuits run alone.

Each circuit of a batch runs through its own context, so whatever the
number of circuits in flight or the use of HIP graphs, its results must be
bit for bit those of the plain per-circuit loop; in FP64 they must also
match the CPU oracle.
"""
import sys

import numpy as np
import pytest

from oracle import dict_oracle as O
from paper_2607_07816_amd import batch as B
from paper_2607_07816_amd import circuits as C
from paper_2607_07816_amd.run import run_circuit

pytestmark = pytest.mark.gpu

FIELDS = ("peak_key", "peak_prob", "n_terms", "gate_steps", "term_updates", "log10_cum_kept")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_items(num=12, seed=11):
    ws = C.batch_workload(num, seed, n_range=(8, 14), depth_range=(2, 5), logk_range=(5, 9))
    return [(c, cfg["K"], 0.0) for c, cfg in ws]


def alone(c, K, p, prec):
    st = run_circuit(c, K=K, p=p, precision=prec, capacity=max(2 * K, 1024))
    key, prob = st.peak()
    out = dict(peak_key=key, peak_prob=prob, n_terms=st.num_terms())
    cnt = st.counters()
    out.update(gate_steps=cnt["gate_steps"], term_updates=cnt["term_updates"],
               log10_cum_kept=st.stats()["log10_cum_kept"])
    st.close()
    return out


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("streams,graph", [(1, 0), (4, 0), (4, 8), (3, 1)])
def test_batch_equals_alone(prec, streams, graph):
    items = small_items()
    say(f"[batch] {len(items)} circuits, {prec}, streams={streams}, graph_steps={graph}")
    res, dt = B.run_batch(items, prec, streams, graph)
    for (c, K, p), r in zip(items, res):
        ref = alone(c, K, p, prec)
        assert r["status"] == 0
        for f in FIELDS:
            assert r[f] == ref[f], (c.name, f, r[f], ref[f])


def test_batch_fp64_matches_oracle():
    # every circuit's final terms, term by term, and its figures against the
    # C oracle run on the same gate list
    import math

    from oracle import c_oracle as CO
    items = small_items(8, seed=12)
    res, _ = B.run_batch(items, "c128", 4, 8, want_terms=True)
    for (c, K, p), r in zip(items, res):
        trace = []
        ko, ao = CO.run_circuit(c.gates, c.truncate_after, K, p, trace=trace)
        ko, ao = CO.sorted_terms(ko, ao)
        key, prob = CO.peak(ko, ao)
        cum = sum(math.log10(t["info"]["fraction"]) for t in trace if t["info"] and t["info"]["dropped"])
        say(f"[batch] {c.name}: K={K} terms {r['n_terms']} oracle {len(ko)} peak {r['peak_key']:#x}")
        assert r["status"] == 0
        assert r["n_terms"] == len(ko)
        assert np.array_equal(r["keys"], ko)
        assert np.abs(r["amps"] - ao).max() <= 1e-12
        assert r["peak_key"] == key
        assert abs(r["peak_prob"] - prob) <= 1e-12
        assert abs(r["log10_cum_kept"] - cum) <= 1e-12
        assert r["gate_steps"] == sum(1 for t in trace if t["info"] is not None)


def test_batch_uneven_sizes_and_order():
    # a mix of sizes; results come back in input order whatever ran first
    items = small_items(6, seed=13) + [(C.workload_small()[0], 1024, 0.0)]
    res, _ = B.run_batch(items[::-1], "c64", 2, 4)
    for (c, K, p), r in zip(items[::-1], res):
        ref = alone(c, K, p, "c64")
        assert r["peak_key"] == ref["peak_key"] and r["n_terms"] == ref["n_terms"]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_replayed_steps_equal_eager_at_every_checkpoint(prec):
    # with graph_steps > 0 the batch runner captures a truncated step once per
    # state of its context and replays it with the next gate; prefixes of one
    # circuit end at different replays, and each prefix's final terms must be
    # bit for bit those of the same prefix run eagerly
    from paper_2607_07816_amd.circuits import Circuit
    base = C.peaked_circuit(14, 6, 0.02, 77, pairs="random", u3_layers=False)
    K = 300
    lengths = [4, 9, 15, 23, 31, 40, 52, len(base.gates)]
    items = []
    for L in lengths:
        c = Circuit(base.n, base.gates[:L], base.truncate_after[:L], base.hidden, base.seed, f"prefix{L}")
        items.append((c, K, 0.0))
    res, _ = B.run_batch(items, prec, 2, 1, want_terms=True)
    for (c, K_, p), r in zip(items, res):
        st = run_circuit(c, K=K_, p=p, precision=prec, capacity=1024)
        k, a = st.read_terms()
        st.close()
        assert r["status"] == 0
        assert np.array_equal(r["keys"], k), c.name
        assert np.array_equal(r["amps"].view(np.uint64), a.view(np.uint64)), c.name
    say(f"[batch] replayed prefixes {lengths} equal the eager runs ({prec})")


@pytest.mark.parametrize("sort", [(20, "11x16"), (20, "8x8"), (12, "11x8")])
def test_batch_sort_shapes_equal_alone(sort):
    # the sort shape the autotuner may choose for small states changes no
    # circuit's result
    items = small_items(8, seed=14)
    res, _ = B.run_batch(items, "c128", 4, 1, sort=sort)
    for (c, K, p), r in zip(items, res):
        ref = alone(c, K, p, "c128")
        assert r["status"] == 0
        for f in FIELDS:
            assert r[f] == ref[f], (c.name, sort, f)
