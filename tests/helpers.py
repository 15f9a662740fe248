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


def check_c64_trajectory(st, circuit, K, p, threads=0, say=print):
    """Run ``circuit`` on the complex64 State ``st`` and check every truncated
    step against one oracle step from the GPU's own state before it (FP32
    amplitudes promoted exactly to FP64): kept fraction within 1e-6, at least
    99% of the oracle's keys kept, per-term error within 1e-5 on them.
    Returns the GPU's kept fractions, step by step."""
    from oracle import c_oracle as CO
    fractions = []
    worst_f = worst_e = 0.0
    worst_c = 1.0
    for (qs, U), tr in zip(circuit.gates, circuit.truncate_after):
        if not tr:
            st.apply_gate(qs, U)
            continue
        kin, ain = st.read_terms()
        st.apply_gate(qs, U)
        st.truncate()
        f = st.stats()["kept_fraction"]
        fractions.append(f)
        kg, ag = st.read_terms()
        kr, ar, info = CO.step(kin, ain, qs, U, K, p, True, threads)
        kr, ar = CO.sorted_terms(kr, ar)
        common, ig, io = np.intersect1d(kg, kr, assume_unique=True, return_indices=True)
        df = abs(f - info["fraction"])
        de = float(np.abs(ag[ig] - ar[io]).max()) if len(common) else 0.0
        cf = len(common) / max(len(kr), 1)
        step = len(fractions) - 1
        assert df <= 1e-6, f"step {step}: kept fraction {f} vs {info['fraction']}"
        assert cf >= 0.99, f"step {step}: common keys {cf}"
        assert de <= 1e-5, f"step {step}: per-term error {de}"
        worst_f, worst_e, worst_c = max(worst_f, df), max(worst_e, de), min(worst_c, cf)
    say(f"  {len(fractions)} steps: worst |d kept fraction| {worst_f:.2e}, worst per-term error {worst_e:.2e}, "
        f"least common-key fraction {worst_c:.6f}")
    return fractions
