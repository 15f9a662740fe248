"""A second, independent CPU form of the gate step: the paper's vectorised
formulation (Sec. IV.A) in numpy - expand every amplitude by its column of U,
derive the new keys with bit operations, then sum contributions per new key
(np.unique + np.add.at as the segmented sum) - against the dictionary oracle."""
import numpy as np
import pytest

from oracle import dict_oracle as O
from paper_2607_07816_amd import circuits as C
from tests.helpers import arrays_to_dict, random_state


def vectorised_apply(keys, amps, qubits, U):
    m = len(qubits)
    d = 1 << m
    mask = np.uint64(sum(1 << q for q in qubits))
    j = np.zeros(keys.shape, dtype=np.int64)
    for t, q in enumerate(qubits):
        j |= ((keys >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << t
    rest = keys & ~mask
    dep = np.zeros(d, dtype=np.uint64)
    for i in range(d):
        for t, q in enumerate(qubits):
            if (i >> t) & 1:
                dep[i] |= np.uint64(1 << q)
    # contribution of amplitude a (pattern j) to output pattern i: U[i, j] * a
    contrib = U[:, j].T * amps[:, None]                  # (N, d)
    newkeys = rest[:, None] | dep[None, :]              # (N, d)
    uk, inv = np.unique(newkeys.reshape(-1), return_inverse=True)
    acc = np.zeros(uk.shape, dtype=np.complex128)
    np.add.at(acc, inv, contrib.reshape(-1))
    nz = acc != 0
    return uk[nz], acc[nz]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_vectorised_equals_oracle(m):
    rng = np.random.default_rng(50 + m)
    keys, amps = random_state(rng, 14, 400)
    for _ in range(4):
        qs = tuple(int(q) for q in rng.choice(14, m, replace=False))
        u = C.haar_unitary(rng, 1 << m)
        vk, va = vectorised_apply(keys, amps, qs, u)
        st = O.apply(arrays_to_dict(keys, amps), qs, u)
        assert set(int(k) for k in vk) == set(st)
        ref = np.array([complex(*st[int(k)]) for k in vk])
        assert np.abs(ref - va).max() <= 1e-13
        keys, amps = vk, va
