"""Pin the dictionary oracle's gate application to the dense 2^n reference."""
import numpy as np
import pytest

from oracle import dense, dict_oracle
from paper_2607_07816_amd import circuits as C


def to_dense(state, n):
    v = np.zeros(1 << n, dtype=np.complex128)
    for k, (re, im) in state.items():
        v[k] = complex(re, im)
    return v


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_random_gates_match_dense(m):
    rng = np.random.default_rng(100 + m)
    n = 8
    psi = dense.zero_state(n)
    st = dict_oracle.ground_state()
    for step in range(10):
        qs = tuple(int(q) for q in rng.choice(n, size=m, replace=False))
        u = C.haar_unitary(rng, 1 << m)
        psi = dense.apply_dense(psi, n, qs, u)
        st = dict_oracle.apply(st, qs, u)
        assert np.abs(to_dense(st, n) - psi).max() <= 1e-12


def test_small_workload_matches_dense_and_peaks_at_hidden():
    c, cfg = C.workload_small()
    psi = dense.run_dense(c.n, c.gates)
    st = dict_oracle.run_circuit(c.gates, c.truncate_after, cfg["K"], cfg["p"])
    assert np.abs(to_dense(st, c.n) - psi).max() <= 1e-12
    k, prob = dict_oracle.peak(st)
    w = np.abs(psi) ** 2
    assert k == int(np.argmax(w)) == c.hidden
    assert prob > 0.5


def test_mixed_gate_sizes_n10():
    rng = np.random.default_rng(5)
    n = 10
    psi = dense.zero_state(n)
    st = dict_oracle.ground_state()
    for step in range(25):
        m = int(rng.integers(1, 4))
        qs = tuple(int(q) for q in rng.choice(n, size=m, replace=False))
        u = C.haar_unitary(rng, 1 << m)
        psi = dense.apply_dense(psi, n, qs, u)
        st = dict_oracle.apply(st, qs, u)
    assert np.abs(to_dense(st, n) - psi).max() <= 1e-12


def test_truncated_steps_match_dense_topk():
    # per step: apply on both, then keep the top K on both and renormalise
    rng = np.random.default_rng(11)
    n, K = 9, 40
    psi = dense.zero_state(n)
    st = dict_oracle.ground_state()
    for step in range(12):
        qs = tuple(int(q) for q in rng.choice(n, size=2, replace=False))
        u = C.haar_su(rng, 4)
        psi = dense.topk_dense(dense.apply_dense(psi, n, qs, u), K)
        st, _ = dict_oracle.truncate(dict_oracle.apply(st, qs, u), K, 0.0)
        assert set(st) == set(dense.to_terms(psi))
        assert np.abs(to_dense(st, n) - psi).max() <= 1e-12
