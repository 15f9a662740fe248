"""Input generator: determinism, unitarity, exact mirror at eps = 0."""
import numpy as np

from paper_2607_07816_amd import circuits as C


def test_deterministic():
    a = C.peaked_circuit(12, 3, 0.05, 7, pairs="random", u3_layers=True)
    b = C.peaked_circuit(12, 3, 0.05, 7, pairs="random", u3_layers=True)
    assert a.hidden == b.hidden
    assert len(a.gates) == len(b.gates)
    for (qa, ua), (qb, ub) in zip(a.gates, b.gates):
        assert qa == qb
        assert np.array_equal(ua, ub)


def test_unitary_and_special():
    rng = np.random.default_rng(0)
    for _ in range(20):
        g = C.haar_su(rng, 4)
        assert np.abs(g.conj().T @ g - np.eye(4)).max() <= 1e-14
        assert abs(np.linalg.det(g) - 1.0) <= 1e-13
    u = C.u3(0.3, 1.1, 2.2)
    assert np.abs(u.conj().T @ u - np.eye(2)).max() <= 1e-15


def test_all_gates_unitary():
    c = C.peaked_circuit(10, 4, 0.05, 1, pairs="brickwork", u3_layers=True, absorb_u3=True)
    for qs, u in c.gates:
        d = 1 << len(qs)
        assert u.shape == (d, d)
        assert np.abs(u.conj().T @ u - np.eye(d)).max() <= 1e-13


def test_eps_zero_inverse_is_exact_dagger():
    c = C.peaked_circuit(8, 2, 0.0, 3, pairs="brickwork", u3_layers=True)
    nx = bin(c.hidden).count("1")
    g = c.gates[: len(c.gates) - nx]
    half = len(g) // 2
    fwd, inv = g[:half], g[half:]
    for (qf, uf), (qi, ui) in zip(fwd, reversed(inv)):
        assert qf == qi
        assert np.abs(ui - uf.conj().T).max() <= 1e-15


def test_shapes_of_named_workloads():
    c, cfg = C.workload_small()
    assert c.n == 10 and cfg["K"] == 1024
    # 4 layers: 5,4,5,4 pairs + 10 U3 each, mirrored, plus X on the hidden bits
    assert len(c.gates) == 2 * (18 + 40) + bin(c.hidden).count("1")
    assert sum(1 for t in c.truncate_after if not t) == bin(c.hidden).count("1")
    c3 = C.peaked_circuit(48, 2, 0.01, 3, pairs="random", u3_layers=False)
    assert all(len(q) == 2 for q, _ in c3.gates[: 2 * 2 * 24])
    for layer in range(2):
        qs = [q for g in c3.gates[layer * 24:(layer + 1) * 24] for q in g[0]]
        assert sorted(qs) == list(range(48))  # a perfect matching per layer
