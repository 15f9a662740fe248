"""Sparse, truncated state-vector simulation of peaked circuits on MI355X.

The hot path (gate application with collision merge, top-k / p-mass
truncation, renormalisation, peak read-out) is HIP for gfx950 behind the C ABI
in include/sts.h (libsts.so). Submodules:

  _lib      - ctypes binding: State (one sparse state on one GPU)
  run       - run_circuit: the plain per-circuit loop
  circuits  - seeded synthetic peaked circuits (inputs)
  build     - compiles libsts.so in-tree with hipcc

Nothing is imported eagerly, so the input generator can be used without a GPU.
"""

__all__ = ["State", "run_circuit"]


def __getattr__(name):
    if name == "State":
        from ._lib import State
        return State
    if name == "run_circuit":
        from .run import run_circuit
        return run_circuit
    raise AttributeError(name)
