"""The dense reference against textbook facts, in the key/qubit convention."""
import numpy as np

from oracle import dense as D
from paper_2607_07816_amd import circuits as C


def basis(n, k):
    v = np.zeros(1 << n, dtype=np.complex128)
    v[k] = 1.0
    return v


def test_x_flips_the_named_bit():
    n = 4
    for q in range(n):
        out = D.apply_dense(basis(n, 0), n, (q,), C.X_GATE)
        assert np.argmax(np.abs(out)) == 1 << q


def test_cnot_truth_table():
    # control = qubits[0], target = qubits[1]; on qubits (1, 3) of 4
    n = 4
    qs = (1, 3)
    for c in (0, 1):
        for t in (0, 1):
            k = (c << 1) | (t << 3) | 0b0101
            out = D.apply_dense(basis(n, k), n, qs, C.CNOT_GATE)
            expect = (c << 1) | ((t ^ c) << 3) | 0b0101
            assert np.argmax(np.abs(out)) == expect
            assert abs(out[expect] - 1.0) == 0.0


def test_hadamard_on_zero():
    out = D.apply_dense(D.zero_state(3), 3, (2,), C.H_GATE)
    s = 1.0 / np.sqrt(2.0)
    assert np.allclose(out[[0, 4]], [s, s], atol=0, rtol=1e-15)
    assert np.count_nonzero(out) == 2


def test_local_bit_order_kron():
    # kron(A, B) puts B on qubits[0]: X on qubits[0] only flips that qubit
    n = 3
    g = np.kron(np.eye(2), C.X_GATE)
    out = D.apply_dense(basis(n, 0), n, (2, 0), g)
    assert np.argmax(np.abs(out)) == 1 << 2


def test_eq3_orientation():
    # Eq. (3): a'_0 = u00 a0 + u01 a1, a'_1 = u10 a0 + u11 a1
    u = np.array([[1 + 2j, 3 - 1j], [0.5j, -2]], dtype=np.complex128)
    a = np.array([0.25 - 1j, 2 + 0.5j])
    out = D.apply_dense(a, 1, (0,), u)
    assert np.allclose(out, [u[0, 0] * a[0] + u[0, 1] * a[1], u[1, 0] * a[0] + u[1, 1] * a[1]], rtol=0, atol=1e-15)
