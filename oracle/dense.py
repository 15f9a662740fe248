"""Dense 2^n state-vector reference (n <= 12), for pinning the oracle.

TEST INFRASTRUCTURE ONLY (see dict_oracle). This is the textbook dense
simulator that the paper contrasts with the sparse approach (Sec. II): the
state is a full complex128 array of length 2^n, and a gate on m qubits is a
tensor contraction of U with the state's qubit axes. It shares no code with
dict_oracle and serves as an independent pin of the gate application.

Basis index k has qubit q at bit q. numpy's reshape to (2,)*n is big-endian,
so axis a of the reshaped tensor is qubit n-1-a.
"""
from __future__ import annotations

import numpy as np


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_dense(psi: np.ndarray, n: int, qubits, U: np.ndarray) -> np.ndarray:
    """psi' = (U on qubits) psi, with local bit t of U's index = qubit qubits[t]."""
    m = len(qubits)
    t = psi.reshape((2,) * n)
    # U as a tensor: axes (i_{m-1}, ..., i_0, j_{m-1}, ..., j_0), big-endian
    ut = np.asarray(U, dtype=np.complex128).reshape((2,) * (2 * m))
    # state axes holding qubits[m-1], ..., qubits[0] (matching U's big-endian j axes)
    axes = [n - 1 - qubits[m - 1 - a] for a in range(m)]
    out = np.tensordot(ut, t, axes=(list(range(m, 2 * m)), axes))
    # out axes: (i_{m-1}..i_0, remaining state axes in order); put i axes back
    out = np.moveaxis(out, list(range(m)), axes)
    return out.reshape(-1)


def run_dense(n: int, gates) -> np.ndarray:
    psi = zero_state(n)
    for qs, u in gates:
        psi = apply_dense(psi, n, qs, u)
    return psi


def to_terms(psi: np.ndarray) -> dict:
    """Nonzero entries as {key: complex}."""
    nz = np.nonzero(psi)[0]
    return {int(k): complex(psi[k]) for k in nz}


def topk_dense(psi: np.ndarray, K: int) -> np.ndarray:
    """Keep the K largest |a|^2 (ties to the smaller index) and renormalise."""
    w = psi.real * psi.real + psi.imag * psi.imag
    order = sorted(range(len(psi)), key=lambda k: (-w[k], k))
    keep = [k for k in order[:K] if w[k] > 0]
    out = np.zeros_like(psi)
    out[keep] = psi[keep]
    return out / np.linalg.norm(out)
