"""The OpenMP twin of the C oracle equals the plain C oracle bit for bit.

The twin splits the same arithmetic over host threads (gate application per
hash bucket of groups, ranking by chunk sorts and merges, exact sums as
partial integer sums); it serves the end-to-end parity runs and the
all-cores CPU baseline, where the plain oracle takes minutes. Thread counts
cover more threads than terms, a prime count (uneven chunks) and powers of
two (the merge rounds).
"""
import numpy as np
import pytest

from oracle import c_oracle as CO
from paper_2607_07816_amd import circuits as C
from tests.helpers import random_state

THREADS = (1, 2, 3, 7, 8)


def by_key(k, a):
    return CO.sorted_terms(k, a)


def same_terms(k1, a1, k2, a2):
    k1, a1 = by_key(k1, a1)
    k2, a2 = by_key(k2, a2)
    return np.array_equal(k1, k2) and np.array_equal(a1.view(np.uint64), a2.view(np.uint64))


@pytest.mark.parametrize("seed", range(3))
def test_apply_mt_bitwise(seed):
    rng = np.random.default_rng(500 + seed)
    for n, N in ((12, 5), (16, 900), (40, 4000)):
        keys, amps = random_state(rng, n, N)
        for m in (1, 2, 3, 5):
            qs = tuple(int(q) for q in rng.choice(n, m, replace=False))
            U = C.haar_unitary(rng, 1 << m)
            k0, a0 = CO.apply(keys, amps, qs, U)
            for t in THREADS:
                k1, a1 = CO.apply(keys, amps, qs, U, threads=t)
                assert same_terms(k0, a0, k1, a1), (n, N, m, t)
    # permutation gates: the term count is kept
    keys, amps = random_state(rng, 20, 3000)
    k1, a1 = CO.apply(keys, amps, (3, 9, 14), C.TOFFOLI_GATE, threads=5)
    assert k1.shape == keys.shape


def test_apply_mt_empty_and_duplicates():
    k, a = CO.apply(np.zeros(0, np.uint64), np.zeros(0, np.complex128), (1,), C.H_GATE, threads=4)
    assert k.shape == (0,)
    with pytest.raises(ValueError):
        CO.apply(np.array([5, 5], np.uint64), np.ones(2, np.complex128), (0,), C.H_GATE, threads=3)


@pytest.mark.parametrize("seed", range(4))
def test_truncate_mt_bitwise(seed):
    rng = np.random.default_rng(600 + seed)
    keys, amps = random_state(rng, 24, 5000, normalise=seed % 2 == 0)
    if seed == 1:
        amps[::4] = amps[0]  # ties, split by key
    for K, p in ((0, 0.9), (1000, 0.0), (1, 0.0), (4999, 0.0), (10 ** 6, 0.0), (700, 0.99), (0, 0.5),
                 (0, 1e-9), (0, 1.0 - 2 ** -40)):
        k0, a0, i0 = CO.truncate(keys, amps, K, p)
        for t in THREADS:
            k1, a1, i1 = CO.truncate(keys, amps, K, p, threads=t)
            # the kept terms in rank order, bit for bit, and the same figures
            assert np.array_equal(k0, k1), (K, p, t)
            assert np.array_equal(a0.view(np.uint64), a1.view(np.uint64))
            assert i0 == i1


def test_truncate_mt_equal_weights_boundary():
    # N equal weights: L_p = ceil(p N); p N integral hits the exact equality
    N = 96
    keys = np.arange(N, dtype=np.uint64) * np.uint64(7)
    amps = np.full(N, 0.25, dtype=np.complex128)
    for p, L in ((0.5, 48), (0.25, 24), (0.3, 29)):
        for t in THREADS:
            k, _, info = CO.truncate(keys, amps, 0, p, threads=t)
            assert np.array_equal(k, keys[:L]) and info["kept"] == L


def test_run_circuit_mt_bitwise():
    c = C.peaked_circuit(14, 3, 0.03, 9, pairs="random", u3_layers=False)
    for K, p in ((256, 0.0), (0, 0.95), (300, 0.999)):
        tr0, tr1 = [], []
        k0, a0 = CO.run_circuit(c.gates, c.truncate_after, K, p, trace=tr0)
        k1, a1 = CO.run_circuit(c.gates, c.truncate_after, K, p, trace=tr1, threads=6)
        assert same_terms(k0, a0, k1, a1)
        assert [t["info"] for t in tr0] == [t["info"] for t in tr1]
