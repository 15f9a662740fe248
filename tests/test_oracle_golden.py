"""Both CPU oracles and the dense reference against hand-derived examples."""
import numpy as np
import pytest

from oracle import c_oracle, dense, dict_oracle
from tests import golden_io
from tests.helpers import arrays_to_dict, dict_to_arrays


@pytest.mark.parametrize("name", golden_io.names())
def test_golden(name):
    n, qubits, U, tin, tout = golden_io.load(name)
    out = dict_oracle.apply(tin, qubits, U)
    assert out == tout  # exact: bitwise equal floats and the same key set
    k, a = dict_to_arrays(tin)
    k2, a2 = c_oracle.apply(k, a, qubits, U)
    assert arrays_to_dict(k2, a2) == tout
    psi = np.zeros(1 << n, dtype=np.complex128)
    for key, (re, im) in tin.items():
        psi[key] = complex(re, im)
    d = dense.to_terms(dense.apply_dense(psi, n, qubits, U))
    assert set(d) == set(tout)
    for key, v in tout.items():
        assert abs(d[key] - complex(*v)) <= 1e-15
