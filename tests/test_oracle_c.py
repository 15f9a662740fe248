"""The C oracle equals the Python dictionary oracle bit for bit."""
import math

import numpy as np
import pytest

from oracle import c_oracle as CO
from oracle import dict_oracle as O
from paper_2607_07816_amd import circuits as C
from tests.helpers import arrays_to_dict, dict_to_arrays, random_state


def same(d, keys, amps):
    return d == arrays_to_dict(keys, amps)


@pytest.mark.parametrize("seed", range(4))
def test_apply_bitwise(seed):
    rng = np.random.default_rng(seed)
    keys, amps = random_state(rng, 16, 500)
    st = arrays_to_dict(keys, amps)
    for m in (1, 2, 3, 4, 5):
        qs = tuple(int(q) for q in rng.choice(16, m, replace=False))
        u = C.haar_unitary(rng, 1 << m)
        k2, a2 = CO.apply(keys, amps, qs, u)
        st2 = O.apply(st, qs, u)
        assert same(st2, k2, a2)
    for g, m in ((C.X_GATE, 1), (C.CNOT_GATE, 2), (C.TOFFOLI_GATE, 3)):
        qs = tuple(int(q) for q in rng.choice(16, m, replace=False))
        k2, a2 = CO.apply(keys, amps, qs, g)
        assert same(O.apply(st, qs, g), k2, a2)
        assert k2.shape[0] == keys.shape[0]


@pytest.mark.parametrize("seed", range(6))
def test_truncate_bitwise(seed):
    rng = np.random.default_rng(100 + seed)
    keys, amps = random_state(rng, 20, 3000, normalise=seed % 2 == 0)
    if seed == 3:
        amps[::3] = amps[0]  # ties
    st = arrays_to_dict(keys, amps)
    for K, p in ((0, 0.0), (1, 0.0), (100, 0.0), (2999, 0.0), (5000, 0.0),
                 (0, 0.5), (0, 0.99), (0, 0.9999999), (200, 0.5), (2000, 0.9), (0, 1.0)):
        ko, ao, info = CO.truncate(keys, amps, K, p)
        st2, info2 = O.truncate(st, K, p)
        assert same(st2, ko, ao), (K, p)
        assert info["kept"] == info2["kept"]
        assert info["W"] == info2["W"] and info["S"] == info2["S"]
        assert info["fraction"] == info2["fraction"]
        assert info["dropped"] == info2["dropped"]


def test_peak_bitwise():
    rng = np.random.default_rng(7)
    keys, amps = random_state(rng, 20, 1000)
    amps[5] = amps[9] = 2.0  # tie for the peak
    assert CO.peak(keys, amps) == O.peak(arrays_to_dict(keys, amps))


def test_exact_sum_matches_fsum():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.random(1000), rng.random(1000) * 1e-20, [5e-324, 2.0 ** -1022, 1e30]])
    rng.shuffle(x)
    assert CO.fsum_nonneg(x) == math.fsum(x.tolist())
    assert CO.fsum_nonneg(np.array([1.0, 2.0 ** -53, 2.0 ** -53])) == 1.0 + 2.0 ** -52
    assert CO.fsum_nonneg(np.array([1.0, 2.0 ** -53])) == 1.0  # tie to even
    assert CO.fsum_nonneg(np.array([1.0, 2.0 ** -53, 2.0 ** -106])) == 1.0 + 2.0 ** -52


def test_circuit_bitwise_small():
    c = C.peaked_circuit(12, 3, 0.03, 17, pairs="random", u3_layers=True, absorb_u3=True)
    st = O.run_circuit(c.gates, c.truncate_after, 200, 0.0)
    k, a = CO.run_circuit(c.gates, c.truncate_after, 200, 0.0)
    assert same(st, k, a)
    st = O.run_circuit(c.gates, c.truncate_after, 0, 0.97)
    k, a = CO.run_circuit(c.gates, c.truncate_after, 0, 0.97)
    assert same(st, k, a)
    assert CO.peak(k, a)[0] == c.hidden
