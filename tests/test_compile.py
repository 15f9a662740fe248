"""Gate reordering and block fusion (Sec. VI.A), pinned by the dense
simulator: the compiled circuit must implement the same unitary, reordering
must keep every qubit's gate sequence, and blocks must respect their size."""
import numpy as np
import pytest

from oracle import dense as D
from paper_2607_07816_amd import circuits as C
from paper_2607_07816_amd import compile as K


def random_gates(rng, n, count, mmax=2):
    gates = []
    for _ in range(count):
        m = int(rng.integers(1, mmax + 1))
        qs = tuple(int(q) for q in rng.choice(n, size=m, replace=False))
        gates.append((qs, C.haar_unitary(rng, 1 << m)))
    return gates


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("max_m,do_reorder", [(2, True), (3, False), (3, True), (4, True), (5, True)])
def test_compiled_circuit_is_the_same_unitary(seed, max_m, do_reorder):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 9))
    gates = random_gates(rng, n, 40, mmax=min(2, max_m))
    c = C.Circuit(n=n, gates=gates, truncate_after=[True] * len(gates), hidden=0, seed=seed, name="r")
    cc = K.compile_circuit(c, max_m, do_reorder)
    assert all(len(qs) <= max_m for qs, _ in cc.gates)
    assert len(cc.gates) <= len(gates)
    # an arbitrary (not basis) input state, so every column of the unitary counts
    psi0 = D.zero_state(n)
    for q in range(n):
        psi0 = D.apply_dense(psi0, n, (q,), C.haar_unitary(rng, 2))
    a, b = psi0.copy(), psi0.copy()
    for qs, u in gates:
        a = D.apply_dense(a, n, qs, u)
    for qs, u in cc.gates:
        b = D.apply_dense(b, n, qs, u)
    assert np.abs(a - b).max() < 1e-12


def test_reorder_keeps_each_qubits_sequence():
    rng = np.random.default_rng(7)
    gates = random_gates(rng, 8, 60)
    new, _ = K.reorder(gates)
    for q in range(8):
        before = [id(u) for qs, u in gates if q in qs]
        after = [id(u) for qs, u in new if q in qs]
        assert before == after


def test_reorder_postpones_new_qubits():
    # after the gate on qubit 0, the later gates on qubit 0 alone introduce
    # nothing new and run before the gate that brings in qubit 5
    mats = [np.eye(2) * (k + 1) for k in range(4)]
    gates = [((0,), mats[0]), ((5,), mats[1]), ((0,), mats[2]), ((0,), mats[3])]
    new, _ = K.reorder(gates)
    assert [id(u) for _, u in new] == [id(mats[0]), id(mats[2]), id(mats[3]), id(mats[1])]


@pytest.mark.parametrize("seed", range(4))
def test_reorder_introduces_qubits_only_when_it_must(seed):
    # at every step: if the chosen gate brings in a new qubit, no gate that
    # was ready at that moment worked on active qubits alone
    rng = np.random.default_rng(200 + seed)
    gates = random_gates(rng, 10, 50)
    new, _ = K.reorder(gates)
    pos = {id(u): k for k, (_, u) in enumerate(new)}
    active, done = set(), set()
    for k, (qs, u) in enumerate(new):
        ready = []
        for j, (gq, gu) in enumerate(gates):
            if id(gu) in done:
                continue
            # ready: every earlier gate sharing a qubit is done
            if all(id(hu) in done for hq, hu in gates[:j] if set(hq) & set(gq)):
                ready.append((gq, gu))
        assert any(gu is u for _, gu in ready)
        if set(qs) - active:
            assert all(set(gq) - active for gq, _ in ready)
        active.update(qs)
        done.add(id(u))


def test_fuse_blocks_and_truncation_flags():
    I2, I4 = np.eye(2), np.eye(4)
    gates = [((0, 1), I4), ((1, 2), I4), ((2, 3), I4), ((0,), I2), ((7,), I2)]
    tr = [True, True, True, False, False]
    fused, ftr = K.fuse(gates, tr, 3)
    assert [qs for qs, _ in fused] == [(0, 1, 2), (2, 3, 0), (7,)]
    assert ftr == [True, True, False]
    with pytest.raises(ValueError):
        K.fuse([((0, 1, 2), np.eye(8))], [True], 2)


def test_embed_matches_kron_order():
    # U on (q_a, q_b) inside block (q_b, q_x, q_a): check one explicit entry
    rng = np.random.default_rng(3)
    U = C.haar_unitary(rng, 4)
    M = K.embed(U, (9, 4), (4, 1, 9))
    # block bit0 = qubit 4 (gate bit1), bit2 = qubit 9 (gate bit0); qubit 1 idle
    for x in range(8):
        j = ((x >> 2) & 1) | (((x >> 0) & 1) << 1)
        for i in range(4):
            y = (x & 0b010) | ((i & 1) << 2) | ((i >> 1) & 1)
            assert M[y, x] == U[i, j]
    assert np.allclose(M.conj().T @ M, np.eye(8))
