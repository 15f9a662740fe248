"""Seeded synthetic peaked circuits (inputs only).

This module draws the gate lists that both the HIP path and the CPU oracle
consume. It holds none of the simulation method's arithmetic: it only builds
unitary matrices from random numbers, so that the two sides receive the same
FP64 matrices in memory.

Construction (mirror circuits). The paper studies peaked circuits, whose
output distribution concentrates on one bit string (Sec. I and Sec. VI); the
circuits it evaluates are not available, so a mirror construction stands in
for them: d forward layers L_1..L_d, then the daggered layers L_d^+..L_1^+
in reverse order with each daggered gate multiplied on the left by
exp(-i*eps*H) for a seeded random Hermitian H, then X on each qubit q with
s_q = 1. With eps = 0 the circuit is exactly X^s, so its output is the basis
state s; with eps > 0 the peak is still at s.

Conventions:
  * qubit q is bit q of the basis key (qubit 0 is the least significant bit);
  * a gate is (qubits, U) with U a 2^m x 2^m complex128 matrix, row-major,
    U[i][j] mapping local pattern j to local pattern i, where local bit t is
    qubit qubits[t] (so np.kron(A, B) puts B on qubits[0]);
  * U3(theta, phi, lam) follows the OpenQASM 2 definition (the gate family of
    the circuit excerpted in Fig. 1).

Random draw order, for reproducibility: s first; then per forward layer the
pairs (brickwork, or a random perfect matching from rng.permutation), one
Haar SU(4) per pair, then (if U3 layers are on) theta, phi, lam for qubits
0..n-1; then per inverse layer (last forward layer first) one random
Hermitian per emitted gate, drawn as the gate is emitted.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[Tuple[int, ...], np.ndarray]


@dataclass
class Circuit:
    """A gate list plus the metadata needed to check it.

    ``truncate_after[g]`` is False only for the final X layer: that layer
    only relabels keys, and a p-mass cut after a pure relabelling would drop
    mass for nothing (each p-mass cut discards up to 1-p again).
    """

    n: int
    gates: List[Gate]
    truncate_after: List[bool]
    hidden: int                      # the hidden bit string s as an integer key
    seed: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_steps(self) -> int:
        return len(self.gates)


# --------------------------------------------------------------------------
# matrices
# --------------------------------------------------------------------------

def haar_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random U(dim): QR of a complex Gaussian with Mezzadri's phase fix."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    q = q * (d / np.abs(d))[None, :]
    return q


def haar_su(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random SU(dim): a Haar unitary divided by a dim-th root of its determinant."""
    q = haar_unitary(rng, dim)
    det = np.linalg.det(q)
    return q / det ** (1.0 / dim)


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """OpenQASM 2 U3(theta, phi, lambda)."""
    c = np.cos(theta / 2.0)
    s = np.sin(theta / 2.0)
    return np.array(
        [[c, -np.exp(1j * lam) * s],
         [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
        dtype=np.complex128,
    )


def random_hermitian(rng: np.random.Generator, dim: int) -> np.ndarray:
    a = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    return (a + a.conj().T) / 2.0


def expm_hermitian(h: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t H) for Hermitian H, through its eigendecomposition."""
    lam, v = np.linalg.eigh(h)
    return (v * np.exp(-1j * t * lam)[None, :]) @ v.conj().T


X_GATE = np.array([[0, 1], [1, 0]], dtype=np.complex128)
H_GATE = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
# 2-qubit gates in the local basis j = bit(qubits[0]) + 2*bit(qubits[1])
CNOT_GATE = np.eye(4, dtype=np.complex128)[[0, 3, 2, 1]]   # control qubits[0], target qubits[1]
SWAP_GATE = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]
CZ_GATE = np.diag([1, 1, 1, -1]).astype(np.complex128)
# Toffoli: controls qubits[0], qubits[1], target qubits[2]
TOFFOLI_GATE = np.eye(8, dtype=np.complex128)[[0, 1, 2, 7, 4, 5, 6, 3]]


# --------------------------------------------------------------------------
# peaked mirror circuits
# --------------------------------------------------------------------------

def _brickwork_pairs(n: int, layer: int) -> List[Tuple[int, int]]:
    start = 0 if layer % 2 == 0 else 1
    return [(q, q + 1) for q in range(start, n - 1, 2)]


def _random_pairs(rng: np.random.Generator, n: int) -> List[Tuple[int, int]]:
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


def peaked_circuit(n: int, depth: int, eps: float, seed: int, *,
                   pairs: str = "brickwork", u3_layers: bool = True,
                   absorb_u3: bool = False, name: str = "") -> Circuit:
    """Mirror peaked circuit.

    pairs:      "brickwork" ((0,1),(2,3),.. then (1,2),(3,4),..) or "random"
                (a random perfect matching per layer).
    u3_layers:  after each forward layer's SU(4)s, a U3 on every qubit.
    absorb_u3:  fold each U3 into the SU(4) of the pair that contains its
                qubit (kron(U3_q1, U3_q0) @ G); qubits in no pair keep a
                stand-alone 1-qubit U3.
    """
    if pairs not in ("brickwork", "random"):
        raise ValueError(pairs)
    rng = np.random.default_rng(seed)
    s_bits = rng.integers(0, 2, n)
    hidden = int(sum(int(b) << q for q, b in enumerate(s_bits)))

    # forward layers: each is an ordered list of gates
    fwd_layers: List[List[Gate]] = []
    for layer in range(depth):
        prs = _brickwork_pairs(n, layer) if pairs == "brickwork" else _random_pairs(rng, n)
        su = [haar_su(rng, 4) for _ in prs]
        u3s = []
        if u3_layers:
            for q in range(n):
                th = rng.uniform(0.0, np.pi)
                ph = rng.uniform(0.0, 2.0 * np.pi)
                la = rng.uniform(0.0, 2.0 * np.pi)
                u3s.append(u3(th, ph, la))
        gates: List[Gate] = []
        if u3_layers and absorb_u3:
            covered = set()
            for (q0, q1), g in zip(prs, su):
                gates.append(((q0, q1), np.kron(u3s[q1], u3s[q0]) @ g))
                covered.update((q0, q1))
            for q in range(n):
                if q not in covered:
                    gates.append(((q,), u3s[q]))
        else:
            for (q0, q1), g in zip(prs, su):
                gates.append(((q0, q1), g))
            for q, u in enumerate(u3s):
                gates.append(((q,), u))
        fwd_layers.append(gates)

    out: List[Gate] = []
    trunc: List[bool] = []
    for gates in fwd_layers:
        for g in gates:
            out.append(g)
            trunc.append(True)
    for gates in reversed(fwd_layers):
        for qs, u in reversed(gates):
            dim = u.shape[0]
            h = random_hermitian(rng, dim)
            ud = expm_hermitian(h, eps) @ u.conj().T
            out.append((qs, ud))
            trunc.append(True)
    for q in range(n):
        if s_bits[q]:
            out.append(((q,), X_GATE.copy()))
            trunc.append(False)
    return Circuit(n=n, gates=out, truncate_after=trunc, hidden=hidden, seed=seed,
                   name=name or f"peaked_n{n}_d{depth}",
                   meta=dict(depth=depth, eps=eps, pairs=pairs, u3_layers=u3_layers,
                             absorb_u3=absorb_u3))


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def workload_small(seed: int = 1) -> Tuple[Circuit, dict]:
    """10 qubits, 4+4 brickwork layers with unfused U3 layers, eps=0.05, FP64,
    K = 1024 = 2^10 (so nothing is ever cut)."""
    c = peaked_circuit(10, 4, 0.05, seed, pairs="brickwork", u3_layers=True,
                       absorb_u3=False, name="peaked10_brick4_eps0.05")
    return c, dict(K=1024, p=0.0, precision="c128")


def workload_24q(seed: int = 2) -> Tuple[Circuit, dict]:
    """24 qubits, 12+12 brickwork layers, U3 folded into the pair gates,
    eps=0.02, top-K with K = 2^20."""
    c = peaked_circuit(24, 12, 0.02, seed, pairs="brickwork", u3_layers=True,
                       absorb_u3=True, name="peaked24_brick12_eps0.02")
    return c, dict(K=1 << 20, p=0.0)


def workload_48q(seed: int = 3) -> Tuple[Circuit, dict]:
    """48 qubits, 16+16 layers of 24 Haar SU(4) on random pairs, eps=0.01,
    cut to min(K = 2^24, L_0.99), complex64 amplitudes."""
    c = peaked_circuit(48, 16, 0.01, seed, pairs="random", u3_layers=False,
                       absorb_u3=False, name="peaked48_rand16_eps0.01")
    return c, dict(K=1 << 24, p=0.99, precision="c64")


def batch_workload(num: int = 256, seed: int = 4, *, n_range=(16, 40), depth_range=(8, 24),
                   eps_range=(0.005, 0.05), logk_range=(12, 20)) -> List[Tuple[Circuit, dict]]:
    """Many independent uneven peaked circuits (random-pair construction)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(num):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.integers(depth_range[0], depth_range[1] + 1))
        eps = float(rng.uniform(eps_range[0], eps_range[1]))
        logk = int(rng.integers(logk_range[0], logk_range[1] + 1))
        cseed = int(rng.integers(0, 2**31 - 1))
        c = peaked_circuit(n, d, eps, cseed, pairs="random", u3_layers=False,
                           name=f"batch{i}_n{n}_d{d}")
        out.append((c, dict(K=1 << logk, p=0.0, precision="c64")))
    return out


def serving_workload(num: int, seed: int = 5, *, n_range=(20, 64), depth_range=(8, 32),
                     eps_range=(0.005, 0.05), logk_range=(14, 22)) -> List[Tuple[Circuit, dict]]:
    """Requests of a serving run: uneven peaked circuits (random-pair
    construction), each cut by top-K or, with probability 1/2, by p = 0.99
    capped at K (p-mass alone can grow without bound)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(num):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.integers(depth_range[0], depth_range[1] + 1))
        eps = float(rng.uniform(eps_range[0], eps_range[1]))
        logk = int(rng.integers(logk_range[0], logk_range[1] + 1))
        pmass = bool(rng.integers(0, 2))
        cseed = int(rng.integers(0, 2**31 - 1))
        c = peaked_circuit(n, d, eps, cseed, pairs="random", u3_layers=False, name=f"req{i}_n{n}_d{d}")
        out.append((c, dict(K=1 << logk, p=0.99 if pmass else 0.0, precision="c64")))
    return out


def gate_arrays(gates: Sequence[Gate]):
    """Flatten a gate list into (m, qubits, U interleaved re/im float64) triples."""
    out = []
    for qs, u in gates:
        u = np.ascontiguousarray(u, dtype=np.complex128)
        out.append((len(qs), np.asarray(qs, dtype=np.int32), u.view(np.float64).reshape(-1).copy()))
    return out
