"""Small conversions shared by the tests (no method arithmetic)."""
import numpy as np


def dict_to_arrays(state):
    keys = np.array(sorted(state), dtype=np.uint64)
    amps = np.array([complex(*state[int(k)]) for k in keys], dtype=np.complex128)
    return keys, amps


def arrays_to_dict(keys, amps):
    return {int(k): (float(a.real), float(a.imag)) for k, a in zip(keys, amps)}


def random_state(rng, n, nterms, normalise=True):
    """Random sparse state with unique keys < 2^n."""
    nterms = min(nterms, 1 << n)
    if n <= 20:
        keys = rng.choice(1 << n, size=nterms, replace=False).astype(np.uint64)
    else:
        ks = set()
        while len(ks) < nterms:
            ks.update(int(x) for x in rng.integers(0, 1 << n, size=nterms - len(ks), dtype=np.uint64))
        keys = np.array(sorted(ks), dtype=np.uint64)
    amps = rng.standard_normal(nterms) + 1j * rng.standard_normal(nterms)
    if normalise:
        amps = amps / np.linalg.norm(amps)
    return keys, amps


def random_gate(rng, n, m, kind="haar"):
    from paper_2607_07816_amd.circuits import haar_unitary
    qs = tuple(int(q) for q in rng.choice(n, size=m, replace=False))
    return qs, haar_unitary(rng, 1 << m)
