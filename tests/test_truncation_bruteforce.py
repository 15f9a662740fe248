"""Truncation rules against brute force, closed forms and invariants."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import dict_oracle as O
from paper_2607_07816_amd import circuits as C
from tests.helpers import arrays_to_dict, random_state


def check_order_invariant(before, after):
    """Kept terms precede dropped ones in (weight desc, key asc)."""
    kept = set(after)
    dropped = [k for k in before if k not in kept]
    if not dropped or not kept:
        return
    wk = {k: O.weight(before[k]) for k in before}
    worst_kept = min(kept, key=lambda k: (wk[k], -k))
    best_dropped = max(dropped, key=lambda k: (wk[k], -k))
    assert wk[worst_kept] >= wk[best_dropped]
    if wk[worst_kept] == wk[best_dropped]:
        assert worst_kept < best_dropped


@pytest.mark.parametrize("seed", range(6))
def test_topk_invariants(seed):
    rng = np.random.default_rng(seed)
    keys, amps = random_state(rng, 12, 200)
    st = arrays_to_dict(keys, amps)
    for K in (1, 7, 100, 199, 200, 500):
        new, info = O.truncate(st, K, 0.0)
        assert len(new) == min(K, len(st))
        check_order_invariant(st, new)
        if K >= len(st):
            assert new == st and not info["dropped"]
        else:
            assert abs(math.fsum(O.weight(a) for a in new.values()) - 1.0) <= 1e-15


def test_pmass_bruteforce_all_subsets():
    rng = np.random.default_rng(42)
    for trial in range(40):
        n = int(rng.integers(1, 11))
        keys, amps = random_state(rng, 6, n, normalise=trial % 2 == 0)
        if trial % 5 == 0:  # force ties in weight
            amps[: n // 2] = amps[0]
        st = arrays_to_dict(keys, amps)
        ws = {k: O.weight(a) for k, a in st.items()}
        W = sum(Fraction(w) for w in ws.values())
        for p in (0.1, 0.5, 0.75, 0.9, 0.99, 0.999999):
            target = Fraction(p) * W
            best = None
            for r in range(1, n + 1):
                if any(sum(Fraction(ws[k]) for k in sub) >= target
                       for sub in itertools.combinations(list(st), r)):
                    best = r
                    break
            new, info = O.truncate(st, 0, p)
            assert len(new) == best
            assert sum(Fraction(ws[k]) for k in new) >= target
            check_order_invariant(st, new)


def test_equal_weights_closed_form():
    # N equal weights: L_p = ceil(p*N) exactly, and the smallest keys survive
    N = 37
    a = (1.0 / math.sqrt(N), 0.0)
    st = {3 * k + 1: a for k in range(N)}
    for p in (0.2, 0.5, 0.51, 0.9):
        new, _ = O.truncate(st, 0, p)
        Lp = math.ceil(Fraction(p) * N)
        assert len(new) == Lp
        assert sorted(new) == sorted(st)[:Lp]


def test_pmass_boundary_equality_is_kept():
    # the prefix mass reaching p*W exactly counts as reaching it (>=): with 40
    # equal weights and p a dyadic fraction, p*N is an integer and L_p = p*N
    N = 40
    a = (0.125, 0.0)
    st = {k: a for k in range(N)}
    for p, L in ((0.5, 20), (0.25, 10), (0.75, 30), (0.025, None)):
        new, _ = O.truncate(st, 0, p)
        if L is None:  # 0.025 is not dyadic: Fraction(0.025)*40 is just above 1
            L = math.ceil(Fraction(p) * N)
        assert len(new) == L
        assert sorted(new) == list(range(L))


def test_hadamard_all_then_topk_keeps_smallest_keys():
    n = 9
    st = O.ground_state()
    for q in range(n):
        st = O.apply(st, (q,), C.H_GATE)
    assert len(st) == 1 << n
    assert len({a for a in st.values()}) == 1  # bitwise equal amplitudes
    for K in (1, 5, 100, 511):
        new, _ = O.truncate(st, K, 0.0)
        assert sorted(new) == list(range(K))


def test_combined_rule_min_of_both():
    # weights 0.4, 0.3, 0.2, 0.1 (times a common factor)
    st = {10: (math.sqrt(0.4), 0.0), 11: (math.sqrt(0.3), 0.0),
          12: (math.sqrt(0.2), 0.0), 13: (math.sqrt(0.1), 0.0)}
    assert len(O.truncate(st, 3, 0.5)[0]) == 2     # p binds
    assert len(O.truncate(st, 1, 0.95)[0]) == 1    # K binds
    assert len(O.truncate(st, 0, 0.95)[0]) == 4    # p alone: all four needed
    assert len(O.truncate(st, 4, 0.0)[0]) == 4     # nothing dropped
    new, info = O.truncate(st, 0, 0.65)
    assert sorted(new) == [10, 11] and info["dropped"]


def test_renormalisation_and_no_op():
    rng = np.random.default_rng(9)
    keys, amps = random_state(rng, 10, 300, normalise=False)
    st = arrays_to_dict(keys, amps)
    new, info = O.truncate(st, 50, 0.0)
    assert abs(math.fsum(O.weight(a) for a in new.values()) - 1.0) <= 1e-15
    assert info["S"] == math.fsum(sorted((O.weight(a) for a in st.values()), reverse=True)[:50])
    same, info2 = O.truncate(st, 1000, 0.0)
    assert same == st and info2["fraction"] == 1.0
    same, _ = O.truncate(st, 0, 0.0)
    assert same == st


def test_peak_ties_go_to_smaller_key():
    st = {9: (0.5, 0.0), 4: (0.0, 0.5), 7: (0.1, 0.0)}
    assert O.peak(st)[0] == 4
