"""Invariants the paper and the mathematics fix, checked on the oracle."""
import math

import numpy as np

from oracle import dict_oracle as O
from paper_2607_07816_amd import circuits as C
from tests.helpers import arrays_to_dict, random_state


def total(st):
    return math.fsum(O.weight(a) for a in st.values())


def test_ground_state_single_term():
    assert O.ground_state() == {0: (1.0, 0.0)}


def test_norm_preserved_without_truncation():
    rng = np.random.default_rng(1)
    st = O.ground_state()
    for _ in range(30):
        qs, u = tuple(int(q) for q in rng.choice(9, 2, replace=False)), C.haar_su(rng, 4)
        st = O.apply(st, qs, u)
    assert abs(total(st) - 1.0) <= 1e-13


def test_hadamard_doubles_terms():
    st = O.apply(O.ground_state(), (3,), C.H_GATE)
    s = C.H_GATE[0, 0].real
    assert st == {0: (s, 0.0), 8: (s, 0.0)}


def perm_check(gate, m):
    rng = np.random.default_rng(7 + m)
    keys, amps = random_state(rng, 8, 60)
    st = arrays_to_dict(keys, amps)
    for _ in range(5):
        qs = tuple(int(q) for q in rng.choice(8, m, replace=False))
        out = O.apply(st, qs, gate)
        assert len(out) == len(st)
        # amplitudes move bit for bit to the permuted keys
        perm = np.argmax(np.abs(gate), axis=0)  # column j -> row perm[j]
        for k, a in st.items():
            j = O.local_index(k, qs)
            nk = (k & ~sum(1 << q for q in qs)) | O.deposit(int(perm[j]), qs)
            assert out[nk] == a
        st = out


def test_permutation_gates_keep_term_count():
    perm_check(C.X_GATE, 1)
    perm_check(C.CNOT_GATE, 2)
    perm_check(C.SWAP_GATE, 2)
    perm_check(C.TOFFOLI_GATE, 3)


def test_identity_is_bitwise_identity():
    rng = np.random.default_rng(3)
    keys, amps = random_state(rng, 10, 100)
    st = arrays_to_dict(keys, amps)
    for m in (1, 2, 3):
        assert O.apply(st, tuple(range(m)), np.eye(1 << m)) == st


def test_gate_then_inverse():
    rng = np.random.default_rng(4)
    keys, amps = random_state(rng, 10, 50)
    st = arrays_to_dict(keys, amps)
    for m in (1, 2, 3, 4):
        qs = tuple(int(q) for q in rng.choice(10, m, replace=False))
        u = C.haar_unitary(rng, 1 << m)
        back = O.apply(O.apply(st, qs, u), qs, u.conj().T)
        for k in set(back) | set(st):
            a = complex(*back.get(k, (0.0, 0.0)))
            b = complex(*st.get(k, (0.0, 0.0)))
            assert abs(a - b) <= 1e-14


def test_eps_zero_peak_is_hidden():
    c = C.peaked_circuit(10, 3, 0.0, 9, pairs="random", u3_layers=False)
    st = O.run_circuit(c.gates, c.truncate_after, 0, 0.0)
    k, prob = O.peak(st)
    assert k == c.hidden
    assert prob >= 1.0 - 1e-12


def test_truncated_run_keeps_peak_small_circuit():
    c = C.peaked_circuit(10, 3, 0.02, 21, pairs="random", u3_layers=False)
    st = O.run_circuit(c.gates, c.truncate_after, 64, 0.0)
    assert len(st) <= 64
    assert O.peak(st)[0] == c.hidden
