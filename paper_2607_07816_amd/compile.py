"""Gate reordering and block fusion (Sec. VI.A).

Two host-side passes over a circuit's gate list, run once before simulation:

reorder(gates)   list scheduling over the circuit's dependency graph (two
                 gates depend on each other when they share a qubit; only
                 independent gates change their relative order). Among the
                 gates whose predecessors are all scheduled, the next one is
                 the gate that brings the fewest not-yet-touched qubits into
                 play (ties: original order), so the set of active qubits -
                 and with it the number of nonzero terms - grows as late as
                 the dependencies allow.

fuse(gates, m)   cuts the (reordered) sequence into blocks of consecutive
                 gates acting on at most m qubits together and multiplies
                 each block into one 2^m x 2^m unitary, so the state is
                 updated, and truncated, once per block instead of once per
                 gate.

The result is an ordinary Circuit whose gates are the fused blocks; a block
is truncated after if any of its gates was.
"""
from __future__ import annotations

import heapq
from dataclasses import replace
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[Tuple[int, ...], np.ndarray]


def reorder(gates: Sequence[Gate], truncate_after: Sequence[bool] = None):
    """Dependency-preserving reordering; returns (gates, truncate_after) in
    the new order."""
    ng = len(gates)
    tr = list(truncate_after) if truncate_after is not None else [True] * ng
    # predecessors: the previous gate on each of a gate's qubits
    last = {}
    preds = [set() for _ in range(ng)]
    succs = [[] for _ in range(ng)]
    for i, (qs, _) in enumerate(gates):
        for q in qs:
            if q in last:
                preds[i].add(last[q])
            last[q] = i
        for p in preds[i]:
            succs[p].append(i)
    waiting = [len(p) for p in preds]
    active = set()
    ready = [i for i in range(ng) if waiting[i] == 0]
    order = []
    # lazy priority queue keyed by (new qubits, index); entries are re-scored
    # when popped, since the active set only grows (scores only fall)
    heap = [(len(set(gates[i][0]) - active), i) for i in ready]
    heapq.heapify(heap)
    while heap:
        score, i = heapq.heappop(heap)
        now = len(set(gates[i][0]) - active)
        if now != score:
            heapq.heappush(heap, (now, i))
            continue
        order.append(i)
        active.update(gates[i][0])
        for s in succs[i]:
            waiting[s] -= 1
            if waiting[s] == 0:
                heapq.heappush(heap, (len(set(gates[s][0]) - active), s))
    assert len(order) == ng
    return [gates[i] for i in order], [tr[i] for i in order]


def embed(U: np.ndarray, gate_qubits: Sequence[int], block_qubits: Sequence[int]) -> np.ndarray:
    """The 2^m matrix acting as U on gate_qubits and as the identity on the
    other qubits of block_qubits (bit t of a local pattern is qubit
    block_qubits[t]; likewise for U and gate_qubits)."""
    m = len(block_qubits)
    pos = [list(block_qubits).index(q) for q in gate_qubits]
    k = len(gate_qubits)
    dim = 1 << m
    M = np.zeros((dim, dim), dtype=np.complex128)
    gmask = sum(1 << p for p in pos)
    for x in range(dim):
        j = 0
        for t, p in enumerate(pos):
            j |= ((x >> p) & 1) << t
        rest = x & ~gmask
        for i in range(1 << k):
            y = rest
            for t, p in enumerate(pos):
                y |= ((i >> t) & 1) << p
            M[y, x] += U[i, j]
    return M


def fuse(gates: Sequence[Gate], truncate_after: Sequence[bool], max_m: int = 3):
    """Greedy blocks of consecutive gates on at most max_m qubits; returns
    (fused gates, truncate_after per block)."""
    if not 1 <= max_m <= 5:
        raise ValueError("blocks of 1..5 qubits")
    out, out_tr = [], []
    blk, blk_q, blk_tr = [], [], False

    def flush():
        nonlocal blk, blk_q, blk_tr
        if not blk:
            return
        qs = tuple(blk_q)
        U = np.eye(1 << len(qs), dtype=np.complex128)
        for gq, gu in blk:
            U = embed(np.asarray(gu, dtype=np.complex128), gq, qs) @ U
        out.append((qs, U))
        out_tr.append(blk_tr)
        blk, blk_q, blk_tr = [], [], False

    for (qs, U), t in zip(gates, truncate_after):
        if len(qs) > max_m:
            raise ValueError(f"a gate on {len(qs)} qubits does not fit blocks of {max_m}")
        union = list(blk_q) + [q for q in qs if q not in blk_q]
        if blk and len(union) > max_m:
            flush()
            union = list(qs)
        blk.append((tuple(qs), U))
        blk_q = union
        blk_tr = blk_tr or bool(t)
    flush()
    return out, out_tr


def compile_circuit(circuit, max_m: int = 3, do_reorder: bool = True):
    """Reorder (optionally) and fuse a circuits.Circuit; returns a new Circuit."""
    gates, tr = list(circuit.gates), list(circuit.truncate_after)
    if do_reorder:
        gates, tr = reorder(gates, tr)
    fused, ftr = fuse(gates, tr, max_m)
    meta = dict(circuit.meta or {})
    meta.update(fused_from=len(circuit.gates), max_m=max_m, reordered=do_reorder)
    return replace(circuit, gates=fused, truncate_after=ftr, name=f"{circuit.name}_fused{max_m}", meta=meta)
