"""The serving runtime (sts_server_*): results of requests served together,
interleaved a few gates at a time and admitted as memory frees, are those of
the same circuits run alone."""
import math
import sys
import threading
import time

import numpy as np
import pytest

from paper_2607_07816_amd import circuits as C
from paper_2607_07816_amd import _lib
from paper_2607_07816_amd.run import run_circuit
from paper_2607_07816_amd.serve import Server

pytestmark = pytest.mark.gpu

FIELDS = ("peak_key", "peak_prob", "n_terms", "gate_steps", "term_updates", "log10_cum_kept")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests(num=10, seed=21):
    ws = C.serving_workload(num, seed, n_range=(8, 16), depth_range=(2, 5), logk_range=(5, 10))
    return [(c, cfg["K"], cfg["p"]) for c, cfg in ws]


def alone(c, K, p):
    st = run_circuit(c, K=K, p=p, precision="c64", capacity=max(2 * min(K, 1 << c.n), 1024))
    key, prob = st.peak()
    cnt = st.counters()
    out = dict(peak_key=key, peak_prob=prob, n_terms=st.num_terms(), gate_steps=cnt["gate_steps"],
               term_updates=cnt["term_updates"], log10_cum_kept=st.stats()["log10_cum_kept"])
    st.close()
    return out


@pytest.mark.parametrize("streams,active,turn", [(1, 1, 1000000), (2, 3, 4), (4, 2, 1)])
def test_served_equals_alone(streams, active, turn):
    items = requests()
    say(f"[serve] {len(items)} requests, streams={streams} active={active} gates/turn={turn}")
    with Server("c64", streams, active, turn, hbm_bytes=1 << 30) as srv:
        tickets = [srv.submit(c, K, p) for c, K, p in items]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["queued"] == 0 and st["active"] == 0 and st["done"] == len(items) and st["bytes_in_use"] == 0
    for (c, K, p), r in zip(items, res):
        ref = alone(c, K, p)
        assert r["status"] == 0
        assert r["latency_seconds"] >= r["seconds"] >= 0 and r["queue_seconds"] >= 0
        for f in FIELDS:
            assert r[f] == ref[f], (c.name, f, r[f], ref[f])


def test_served_fp64_matches_oracle():
    # a served FP64 mix (interleaved a few gates at a time, several streams):
    # every request's final terms and figures equal the C oracle's on the
    # same gate list
    from oracle import c_oracle as CO
    items = requests(8, seed=24)
    with Server("c128", 3, 2, 3, hbm_bytes=1 << 30) as srv:
        tickets = [srv.submit(c, K, p, want_terms=True) for c, K, p in items]
        res = [srv.wait(t) for t in tickets]
    for (c, K, p), r in zip(items, res):
        trace = []
        ko, ao = CO.run_circuit(c.gates, c.truncate_after, K, p, trace=trace)
        ko, ao = CO.sorted_terms(ko, ao)
        key, prob = CO.peak(ko, ao)
        cum = sum(math.log10(t["info"]["fraction"]) for t in trace if t["info"] and t["info"]["dropped"])
        say(f"[serve] {c.name}: K={K} p={p} terms {r['n_terms']} oracle {len(ko)} peak {r['peak_key']:#x}")
        assert r["status"] == 0
        assert r["n_terms"] == len(ko)
        assert np.array_equal(r["keys"], ko)
        assert np.abs(r["amps"] - ao).max() <= 1e-12
        assert r["peak_key"] == key and abs(r["peak_prob"] - prob) <= 1e-12
        assert abs(r["log10_cum_kept"] - cum) <= 1e-12


def test_admission_waits_for_memory():
    # a budget that holds about two requests' contexts at a time: all are
    # still served, in order of admission, with nothing left in use
    ws = C.serving_workload(8, 22, n_range=(14, 14), depth_range=(2, 4), logk_range=(10, 10))
    items = [(c, cfg["K"], cfg["p"]) for c, cfg in ws]
    needs = {_lib.required_bytes(max(2 * min(K, 1 << c.n), 1024), _lib.STS_C64) for c, K, _ in items}
    assert len(needs) == 1  # every request needs the same block
    need = needs.pop()
    with Server("c64", 4, 4, 2, hbm_bytes=2 * need + 4096) as srv:
        tickets = [srv.submit(c, K, p) for c, K, p in items]
        peak_active = 0
        while srv.stats()["done"] < len(items):
            peak_active = max(peak_active, srv.stats()["active"])
            time.sleep(0.001)
        res = [srv.wait(t) for t in tickets]
    say(f"[serve] most requests active at once: {peak_active}")
    assert peak_active <= 2
    for (c, K, p), r in zip(items, res):
        assert r["status"] == 0 and r["peak_key"] == alone(c, K, p)["peak_key"]


def test_submission_from_threads_and_errors():
    items = requests(6, seed=23)
    with Server("c64", 2, 2, 3, hbm_bytes=1 << 30) as srv:
        out = {}

        def client(i):
            c, K, p = items[i]
            out[i] = srv.wait(srv.submit(c, K, p))

        th = [threading.Thread(target=client, args=(i,)) for i in range(len(items))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        with pytest.raises(_lib.StsError):
            srv.wait(987654321)  # unknown ticket
    for i, (c, K, p) in enumerate(items):
        assert out[i]["peak_key"] == alone(c, K, p)["peak_key"]
    # a request whose context can never fit is refused at submission
    with Server("c64", 1, 1, 1, hbm_bytes=1 << 20) as srv:
        c, K, p = items[0]
        with pytest.raises(_lib.CapacityError):
            srv.submit(c, K, p)
