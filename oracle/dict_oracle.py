"""Dictionary-of-terms FP64 oracle for the sparse, truncated state vector.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the benchmark's CPU
baseline leg use it.

This is a plain, slow, obviously correct CPU implementation of what the
method computes, in plain Python floats (IEEE binary64, each operation
rounded once, no fused multiply-add), for small cases. A state is a dict
{key: (re, im)} holding only nonzero amplitudes (Sec. I, ground state as a
single term). Qubit q is bit q of the key.

  apply()    - Eq. (3) generalised to m qubits (Sec. IV.A): every amplitude
               multiplies the column of U picked by its local bit pattern,
               the new keys follow from bit operations, and contributions to
               the same new key are summed (the segmented sum of Sec. IV.A).
  truncate() - Sec. III and Sec. IV.B: order terms by decreasing |a|^2,
               keep a prefix chosen by p-mass first, then top-k, and
               renormalise.
  peak()     - the most probable bit string (Sec. I, Sec. V).

Readings where the paper is silent (each also listed in the design notes):
  * local pattern index j = sum_t bit(key, q_t) * 2^t (q_0 least significant);
  * the sum over contributions runs over present j in ascending order,
    starting from +0.0, with complex products (ur*vr - ui*vi, ur*vi + ui*vr);
  * a term is dropped only when both parts are exactly zero;
  * ties in |a|^2 are broken by ascending key;
  * p-mass keeps the shortest prefix whose exact mass is >= p * W, with W the
    current total; p <= 0 or p >= 1 turns it off; K = 0 turns top-k off;
  * when nothing is dropped the state is left bitwise unchanged;
  * the kept mass S is the correctly rounded sum of the kept weights, and the
    scale is fl(1 / fl(sqrt(S))), applied to each component with one rounding.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

Amp = Tuple[float, float]
State = Dict[int, Amp]


def ground_state() -> State:
    """The all-zeros basis state as a single term (Sec. I)."""
    return {0: (1.0, 0.0)}


def local_index(key: int, qubits: Sequence[int]) -> int:
    """Bit pattern of ``key`` on the gate's qubits: bit t of j is bit qubits[t] of key."""
    j = 0
    for t, q in enumerate(qubits):
        j |= ((key >> q) & 1) << t
    return j


def deposit(i: int, qubits: Sequence[int]) -> int:
    """Inverse of local_index on the gate's bits: bit t of i goes to bit qubits[t]."""
    k = 0
    for t, q in enumerate(qubits):
        k |= ((i >> t) & 1) << q
    return k


def apply(state: State, qubits: Sequence[int], U) -> State:
    """Apply the 2^m x 2^m matrix U (U[i][j] complex) on ``qubits``.

    Group the terms by their bits outside the gate (all members of a group
    differ only on the gate's qubits, Sec. IV.A), then for each group form
    new_i = sum_j U[i][j] * a_j over the members present.
    """
    m = len(qubits)
    if len(set(qubits)) != m:
        raise ValueError("duplicate qubits")
    mask = 0
    for q in qubits:
        mask |= 1 << q
    groups: Dict[int, Dict[int, Amp]] = {}
    for key, a in state.items():
        rest = key & ~mask
        groups.setdefault(rest, {})[local_index(key, qubits)] = a
    out: State = {}
    dim = 1 << m
    for rest, members in groups.items():
        js = sorted(members)
        for i in range(dim):
            acc_r = 0.0
            acc_i = 0.0
            for j in js:
                vr, vi = members[j]
                u = U[i][j]
                ur, ui = float(u.real), float(u.imag)
                tr = ur * vr - ui * vi
                ti = ur * vi + ui * vr
                acc_r = acc_r + tr
                acc_i = acc_i + ti
            if acc_r != 0.0 or acc_i != 0.0:
                out[rest | deposit(i, qubits)] = (acc_r, acc_i)
    return out


def weight(a: Amp) -> float:
    """|a|^2 = fl(fl(re*re) + fl(im*im))."""
    return a[0] * a[0] + a[1] * a[1]


def ranked(state: State) -> List[Tuple[int, Amp, float]]:
    """Terms in the total order (weight descending, key ascending)."""
    items = [(k, a, weight(a)) for k, a in state.items()]
    items.sort(key=lambda t: (-t[2], t[0]))
    return items


def _mass_on(p: float) -> bool:
    return 0.0 < p < 1.0


def cut_length(weights_desc: Sequence[float], K: int, p: float) -> int:
    """Number of terms kept: p-mass first, then top-k (Sec. III).

    L_p is the shortest prefix whose exact mass reaches p * W (W the current
    total, exact rational arithmetic); the kept count is min(L_p, K, N).
    """
    n = len(weights_desc)
    lp = n
    if _mass_on(p):
        total = sum((Fraction(w) for w in weights_desc), Fraction(0))
        target = Fraction(p) * total
        run = Fraction(0)
        for idx, w in enumerate(weights_desc):
            run += Fraction(w)
            if run >= target:
                lp = idx + 1
                break
    keep = lp
    if K > 0:
        keep = min(keep, K)
    return min(keep, n)


def truncate(state: State, K: int, p: float):
    """Truncate and renormalise. Returns (new_state, info).

    info = dict(W=fsum of all weights, S=fsum of kept weights, kept=L,
                fraction=S/W, dropped=bool).
    """
    items = ranked(state)
    ws = [w for _, _, w in items]
    n = len(items)
    W = math.fsum(ws)
    L = cut_length(ws, K, p)
    if L >= n:
        return dict(state), dict(W=W, S=W, kept=n, fraction=1.0, dropped=False)
    S = math.fsum(ws[:L])
    scale = 1.0 / math.sqrt(S)
    new: State = {}
    for k, a, _ in items[:L]:
        new[k] = (a[0] * scale, a[1] * scale)
    return new, dict(W=W, S=S, kept=L, fraction=S / W, dropped=True)


def peak(state: State) -> Tuple[int, float]:
    """Most probable key (ties to the smallest key) and its probability w / sum(w)."""
    items = ranked(state)
    W = math.fsum(w for _, _, w in items)
    k, _, w = items[0]
    return k, w / W


def run_circuit(gates, truncate_after, K: int, p: float, state: State | None = None,
                trace: list | None = None) -> State:
    """Apply each gate, truncating after the gates flagged in ``truncate_after``."""
    st = ground_state() if state is None else dict(state)
    for (qs, U), tr in zip(gates, truncate_after):
        n_in = len(st)
        st = apply(st, qs, U)
        info = None
        if tr and (K > 0 or _mass_on(p)):
            st, info = truncate(st, K, p)
        if trace is not None:
            trace.append(dict(n_in=n_in, n_out=len(st), info=info))
    return st
