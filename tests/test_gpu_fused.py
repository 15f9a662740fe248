"""Fused circuits (blocks of 3 to 5 qubits, Sec. VI.A) on the GPU against
the FP64 oracle running the same fused gate list."""
import sys

import numpy as np
import pytest

from oracle import c_oracle as CO
from paper_2607_07816_amd import circuits as C
from paper_2607_07816_amd import compile as K
from paper_2607_07816_amd.run import run_circuit

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("max_m", [3, 4, 5])
@pytest.mark.parametrize("K_", [1024, 48])
def test_fused_small_circuit_fp64(max_m, K_):
    c, _ = C.workload_small()
    cc = K.compile_circuit(c, max_m)
    say(f"[fused] {c.name}: {len(c.gates)} gates -> {len(cc.gates)} blocks of <= {max_m} qubits, K={K_}")
    st = run_circuit(cc, K=K_, p=0.0, precision="c128", capacity=max(K_ << max_m, 4096))
    kg, ag = st.read_terms()
    key, prob = st.peak()
    st.close()
    ko, ao = CO.run_circuit(cc.gates, cc.truncate_after, K_, 0.0)
    ko, ao = CO.sorted_terms(ko, ao)
    assert np.array_equal(kg, ko)
    assert np.abs(ag - ao).max() <= 1e-12
    w = ao.real ** 2 + ao.imag ** 2
    best = np.lexsort((ko, -w))[0]
    assert key == int(ko[best])


def test_fused_24q_c64_same_peak():
    c, cfg = C.workload_24q()
    cc = K.compile_circuit(c, 3)
    K_ = 1 << 14
    st = run_circuit(cc, K=K_, p=0.0, precision="c64", capacity=K_ << 3)
    key, prob = st.peak()
    st.close()
    ko, ao = CO.run_circuit(cc.gates, cc.truncate_after, K_, 0.0)
    w = ao.real ** 2 + ao.imag ** 2
    best = int(ko[np.lexsort((ko, -w))[0]])
    say(f"[fused] 24q blocks {len(cc.gates)}: gpu peak {key:#x} oracle {best:#x} hidden {c.hidden:#x}")
    assert key == best
