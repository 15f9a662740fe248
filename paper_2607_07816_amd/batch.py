"""Batches of independent circuits on one GPU (sts_batch_run) and a small
autotuner for the batch runner's launch configuration.

A batch item is (circuit, K, p). Every circuit runs through its own context,
exactly as it would alone; the batch only decides how many run at once
(`streams`), whether truncated gate steps are captured into HIP graphs
and replayed with the next gate (`graph_steps` > 0), and which shape the
grouping sort takes for small states (digit width and tile, `sort`). None of
these changes a result.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import time
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib


class _Packed:
    """A circuit flattened into the arrays sts_circuit points at (kept alive
    here). With want_terms, room for the final terms as well (at most
    min(K, 2^n) of them, or 2^n without top-k)."""

    MAX_OUT = 1 << 26

    def __init__(self, circuit, K: int, p: float, want_terms: bool = False):
        self.m = np.ascontiguousarray([len(qs) for qs, _ in circuit.gates], dtype=np.int32)
        self.q = np.ascontiguousarray([q for qs, _ in circuit.gates for q in qs], dtype=np.int32)
        self.u = np.ascontiguousarray(np.concatenate(
            [np.ascontiguousarray(u, dtype=np.complex128).reshape(-1).view(np.float64) for _, u in circuit.gates])
            if circuit.gates else np.zeros(0), dtype=np.float64)
        self.t = np.ascontiguousarray(circuit.truncate_after, dtype=np.uint8)
        self.keys = self.amps = None
        cap, kp, ap = 0, None, None
        if want_terms:
            full = 1 << min(int(circuit.n), 62)
            cap = min(int(K), full) if K else full
            if cap > self.MAX_OUT:
                raise ValueError(f"final state of up to {cap} terms is too large to return")
            self.keys = np.zeros(max(cap, 1), dtype=np.uint64)
            self.amps = np.zeros(max(cap, 1), dtype=np.complex128)
            kp, ap = self.keys.ctypes.data, self.amps.ctypes.data
        self.c = _lib.Circuit(int(circuit.n), int(K), float(p), len(circuit.gates), self.m.ctypes.data,
                              self.q.ctypes.data, self.u.ctypes.data, self.t.ctypes.data, cap, kp, ap)

    def terms(self, n: int):
        """The final terms (ascending keys) once the circuit has finished."""
        return self.keys[:n].copy(), self.amps[:n].copy()


def pack(items: Sequence[Tuple[object, int, float]], want_terms: bool = False) -> List[_Packed]:
    return [_Packed(c, K, p, want_terms) for c, K, p in items]


def run_batch(items, precision="c64", streams: int = 8, graph_steps: int = 0, packed=None,
              want_terms: bool = False, sort: Tuple[int, str] = (0, "8x16")) -> Tuple[list, float]:
    """Run every (circuit, K, p) of `items`; returns (per-circuit result
    dicts in input order, wall seconds of the whole batch). With want_terms
    each result also holds the final 'keys' and 'amps' (ascending keys).
    sort = (small_log2, shape): states of at most 2^small_log2 terms are
    grouped with that sort shape (sts_set_sort_shape)."""
    L = _lib.load()
    packed = packed if packed is not None else pack(items, want_terms)
    n = len(packed)
    arr = (_lib.Circuit * max(n, 1))(*[pk.c for pk in packed])
    res = (_lib.CircuitResult * max(n, 1))()
    shape = _lib.SORT_SHAPES[sort[1]] if isinstance(sort[1], str) else int(sort[1])
    cfg = _lib.BatchConfig(_lib._prec(precision), int(streams), int(graph_steps), int(sort[0]), shape)
    t0 = time.perf_counter()
    rc = L.sts_batch_run(n, arr, ctypes.byref(cfg), res)
    dt = time.perf_counter() - t0
    _lib._check(rc, "sts_batch_run")
    out = []
    for i in range(n):
        r = res[i]
        d = dict(status=r.status, peak_key=int(r.peak_key), peak_prob=r.peak_prob, n_terms=int(r.n_terms),
                 gate_steps=int(r.gate_steps), term_updates=int(r.term_updates),
                 log10_cum_kept=r.log10_cum_kept, seconds=r.seconds)
        if packed[i].keys is not None:
            d["keys"], d["amps"] = packed[i].terms(d["n_terms"])
        out.append(d)
    return out, dt


DEFAULT_CANDIDATES = tuple((s, g) for s in (4, 8, 16, 32, 48) for g in (0, 16))
# grouping-sort policies tried at the best (streams, graph) setting: states of
# at most 2^small_log2 terms sorted with the shape (sts_set_sort_shape)
DEFAULT_SORTS = ((0, "8x16"), (20, "11x16"), (20, "8x8"), (20, "11x8"))


def batch_signature(items, precision="c64") -> str:
    """Key of a batch's shape for the autotuner's cache: the precision, the
    number of circuits and a histogram of (qubits, log2 K, gates / 8, p on)
    over them. Batches of the same mix of sizes share a configuration."""
    hist = {}
    for c, K, p in items:
        k = (int(c.n), int(K).bit_length(), len(c.gates) // 8, bool(0.0 < p < 1.0))
        hist[k] = hist.get(k, 0) + 1
    body = json.dumps([precision, len(items), sorted([list(k) + [v] for k, v in hist.items()])])
    return hashlib.sha256(body.encode()).hexdigest()[:32]


def _load_cache(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def autotune(items, precision="c64", sample: Optional[Sequence[int]] = None,
             candidates: Iterable[Tuple[int, int]] = DEFAULT_CANDIDATES, repeats: int = 1,
             cache: Optional[str] = None, sorts: Iterable[Tuple[int, str]] = DEFAULT_SORTS):
    """Time each (streams, graph_steps) candidate on a sample of the batch,
    then each grouping-sort policy (small_log2, shape) at the best of them,
    and return (best config (streams, graph_steps, small_log2, shape),
    {config: seconds}). The sample keeps the batch's mix: by default every
    fourth circuit. The sort policy chooses the sort's digit width and tile
    by the state's size (log2 of its term bound).

    With `cache` (a JSON file path), a batch whose signature (batch_signature)
    and candidate lists were tuned before returns the stored choice and
    timings without running anything; a new result is added to the file."""
    candidates = [tuple(int(x) for x in c) for c in candidates]
    sorts = [(int(a), str(b)) for a, b in sorts]
    key = (batch_signature(items, precision) + ":" + ",".join(f"{s}/{g}" for s, g in candidates) + ":" +
           ",".join(f"{a}/{b}" for a, b in sorts))
    if cache:
        hit = _load_cache(cache).get(key)
        if hit:
            timings = {tuple(t[0]): float(t[1]) for t in hit["timings"]}
            return tuple(hit["choice"]), timings
    idx = list(sample) if sample is not None else list(range(0, len(items), 4))
    sub = [items[i] for i in idx]
    packed = pack(sub)

    def timed(streams, graph, sort):
        best = None
        for _ in range(repeats):
            _, dt = run_batch(sub, precision, streams, graph, packed=packed, sort=sort)
            best = dt if best is None else min(best, dt)
        return best

    timings = {}
    default_sort = sorts[0] if sorts else (0, "8x16")
    for s_, g_ in candidates:
        timings[(s_, g_) + default_sort] = timed(s_, g_, default_sort)
    best = min(timings, key=timings.get)
    for sort in sorts[1:]:
        timings[best[:2] + sort] = timed(best[0], best[1], sort)
    choice = min(timings, key=timings.get)
    if cache:
        data = _load_cache(cache)
        data[key] = {"choice": list(choice), "timings": [[list(k), v] for k, v in timings.items()]}
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(tmp, cache)
    return choice, timings
