"""The plain per-circuit loop: apply each gate, truncate after it (the
simulation loop of Sec. VI.A: update by the unitary, then truncate), and
read out the peak (Sec. V: only the final result crosses to the host)."""
from __future__ import annotations

from typing import Optional

from ._lib import State


def run_circuit(circuit, K: int = 0, p: float = 0.0, precision: str = "c128", capacity: Optional[int] = None,
                device: int = 0, stream=None, state: Optional[State] = None, trace: Optional[list] = None):
    """Run ``circuit`` (circuits.Circuit) on the GPU; returns the State.

    Truncation follows every gate flagged in circuit.truncate_after (all but
    the final X layer) when a rule (K or p) is set.
    """
    st = state or State(circuit.n, K=K, p=p, precision=precision, capacity=capacity, device=device, stream=stream)
    rule = K > 0 or 0.0 < p < 1.0
    for (qs, U), tr in zip(circuit.gates, circuit.truncate_after):
        st.apply_gate(qs, U)
        if tr and rule:
            st.truncate()
            if trace is not None:
                trace.append(st.stats())
    return st
