"""ctypes wrapper around the plain-C FP64 oracle (oracle/sts_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

States are passed as (keys uint64[n], amps complex128[n]) numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sts_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-fopenmp"]

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64 = ctypes.c_uint64
        p = ctypes.c_void_p
        L.orc_apply.argtypes = [u64, p, p, ctypes.c_int, p, p, u64, p, p, p]
        L.orc_apply.restype = ctypes.c_int
        L.orc_truncate.argtypes = [u64, p, p, u64, ctypes.c_double, p, p, p, p, p]
        L.orc_truncate.restype = ctypes.c_int
        L.orc_peak.argtypes = [u64, p, p, p, p]
        L.orc_peak.restype = ctypes.c_int
        L.orc_weight_sum.argtypes = [u64, p]
        L.orc_weight_sum.restype = ctypes.c_double
        L.orc_fsum_nonneg.argtypes = [u64, p]
        L.orc_fsum_nonneg.restype = ctypes.c_double
        L.orc_apply_mt.argtypes = L.orc_apply.argtypes + [ctypes.c_int]
        L.orc_apply_mt.restype = ctypes.c_int
        L.orc_truncate_mt.argtypes = L.orc_truncate.argtypes + [ctypes.c_int]
        L.orc_truncate_mt.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def ground_state() -> Tuple[np.ndarray, np.ndarray]:
    return np.zeros(1, dtype=np.uint64), np.ones(1, dtype=np.complex128)


def host_threads() -> int:
    """Host cores this process may use (its CPU affinity, else os.cpu_count())."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def apply(keys: np.ndarray, amps: np.ndarray, qubits, U: np.ndarray, threads: int = 0):
    """Apply U on qubits; returns new (keys, amps) in group order.
    threads = 0: the plain single-threaded oracle; threads >= 1: its OpenMP
    twin on that many threads (bitwise the same terms, in another order)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    amps = np.ascontiguousarray(amps, dtype=np.complex128)
    n = keys.shape[0]
    m = len(qubits)
    qs = np.ascontiguousarray(qubits, dtype=np.int32)
    u = np.ascontiguousarray(U, dtype=np.complex128)
    cap = max(1, n << m)
    ko = np.empty(cap, dtype=np.uint64)
    ao = np.empty(cap, dtype=np.complex128)
    nout = ctypes.c_uint64(0)
    args = (n, _ptr(keys), _ptr(amps), m, _ptr(qs), _ptr(u), cap, ctypes.byref(nout), _ptr(ko), _ptr(ao))
    rc = lib().orc_apply_mt(*args, int(threads)) if threads else lib().orc_apply(*args)
    if rc != 0:
        raise ValueError(f"orc_apply failed ({rc})")
    k = nout.value
    return ko[:k].copy(), ao[:k].copy()


def truncate(keys: np.ndarray, amps: np.ndarray, K: int, p: float, threads: int = 0):
    """Returns (keys, amps, info); info as in dict_oracle.truncate.
    threads as in apply (the result is the same either way)."""
    keys = np.array(keys, dtype=np.uint64, copy=True)
    amps = np.array(amps, dtype=np.complex128, copy=True)
    n = keys.shape[0]
    nout = ctypes.c_uint64(0)
    W = ctypes.c_double(0)
    S = ctypes.c_double(0)
    f = ctypes.c_double(0)
    d = ctypes.c_int(0)
    args = (n, _ptr(keys), _ptr(amps), int(K), float(p), ctypes.byref(nout), ctypes.byref(W), ctypes.byref(S),
            ctypes.byref(f), ctypes.byref(d))
    rc = lib().orc_truncate_mt(*args, int(threads)) if threads else lib().orc_truncate(*args)
    if rc != 0:
        raise RuntimeError("orc_truncate failed")
    L = nout.value
    info = dict(W=W.value, S=S.value, kept=L, fraction=f.value, dropped=bool(d.value))
    return keys[:L].copy(), amps[:L].copy(), info


def peak(keys: np.ndarray, amps: np.ndarray):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    amps = np.ascontiguousarray(amps, dtype=np.complex128)
    k = ctypes.c_uint64(0)
    pr = ctypes.c_double(0)
    rc = lib().orc_peak(keys.shape[0], _ptr(keys), _ptr(amps), ctypes.byref(k), ctypes.byref(pr))
    if rc != 0:
        raise ValueError("empty state")
    return int(k.value), pr.value


def weight_sum(amps: np.ndarray) -> float:
    amps = np.ascontiguousarray(amps, dtype=np.complex128)
    return lib().orc_weight_sum(amps.shape[0], _ptr(amps))


def fsum_nonneg(x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_fsum_nonneg(x.shape[0], _ptr(x))


def step(keys, amps, qubits, U, K: int, p: float, do_truncate: bool = True, threads: int = 0):
    """One gate step: apply, then (optionally) truncate."""
    k2, a2 = apply(keys, amps, qubits, U, threads)
    info = None
    if do_truncate and (K > 0 or 0.0 < p < 1.0):
        k2, a2, info = truncate(k2, a2, K, p, threads)
    return k2, a2, info


def run_circuit(gates, truncate_after, K: int, p: float, state=None, trace=None, threads: int = 0):
    keys, amps = ground_state() if state is None else state
    for (qs, U), tr in zip(gates, truncate_after):
        n_in = keys.shape[0]
        keys, amps, info = step(keys, amps, qs, U, K, p, tr, threads)
        if trace is not None:
            trace.append(dict(n_in=n_in, n_out=keys.shape[0], info=info))
    return keys, amps


def sorted_terms(keys: np.ndarray, amps: np.ndarray):
    """(keys, amps) sorted by key, for comparisons."""
    o = np.argsort(keys, kind="stable")
    return keys[o], amps[o]
