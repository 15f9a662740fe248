"""ctypes binding of libsts (include/sts.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI. PyTorch supplies the device memory (one uint8
arena tensor per state) and the stream. There is no CPU fallback: without
the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsts.so")

STS_OK, STS_E_ARG, STS_E_NOMEM, STS_E_CAPACITY, STS_E_HIP, STS_E_STATE = 0, -1, -2, -3, -4, -5
STS_C128, STS_C64 = 0, 1

# every symbol include/sts.h declares
EXPORTS = (
    "sts_required_bytes", "sts_init", "sts_apply_gate", "sts_truncate", "sts_peak",
    "sts_num_terms", "sts_read_terms", "sts_load_terms", "sts_stats", "sts_counters",
    "sts_profile", "sts_kernel_time", "sts_free", "sts_strerror", "sts_batch_run",
    "sts_server_create", "sts_server_submit", "sts_server_wait", "sts_server_stats", "sts_server_destroy",
    "sts_step_static", "sts_set_sort_shape",
)
SORT_SHAPES = {"8x16": 0, "8x8": 1, "11x16": 2, "11x8": 3}  # sts_sort_shape
STATIC_MAX_TERMS = 65536  # STS_STATIC_MAX_TERMS

KERNEL_KINDS = ("radix_hist", "radix_scan", "radix_pass", "group_hist", "pick1", "group_extract",
                "side_hist", "final", "group_emit", "side_extract", "tile_kept", "tile_scan", "sample")


class Circuit(ctypes.Structure):
    """sts_circuit: one circuit of a batch (flattened gate arrays)."""
    _fields_ = [("n_qubits", ctypes.c_int), ("max_terms", ctypes.c_uint64), ("mass", ctypes.c_double),
                ("n_gates", ctypes.c_uint64), ("gate_m", ctypes.c_void_p), ("gate_qubits", ctypes.c_void_p),
                ("gate_U", ctypes.c_void_p), ("truncate_after", ctypes.c_void_p),
                ("out_cap", ctypes.c_uint64), ("out_keys", ctypes.c_void_p), ("out_amps", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    """sts_batch_config."""
    _fields_ = [("precision", ctypes.c_int), ("n_streams", ctypes.c_int), ("graph_steps", ctypes.c_int),
                ("sort_small_log2", ctypes.c_int), ("sort_shape", ctypes.c_int)]


class CircuitResult(ctypes.Structure):
    """sts_circuit_result."""
    _fields_ = [("status", ctypes.c_int), ("peak_key", ctypes.c_uint64), ("peak_prob", ctypes.c_double),
                ("n_terms", ctypes.c_uint64), ("gate_steps", ctypes.c_uint64), ("term_updates", ctypes.c_uint64),
                ("log10_cum_kept", ctypes.c_double), ("seconds", ctypes.c_double),
                ("queue_seconds", ctypes.c_double), ("latency_seconds", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    """sts_server_config."""
    _fields_ = [("precision", ctypes.c_int), ("n_streams", ctypes.c_int), ("max_active", ctypes.c_int),
                ("gates_per_turn", ctypes.c_int), ("hbm_bytes", ctypes.c_uint64)]


class StsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class CapacityError(StsError):
    pass


_lib = None


def load() -> ctypes.CDLL:
    """Load libsts.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2607_07816_amd/build.py (hipcc, gfx950)")
    # torch first: its HIP runtime has the same soname as the one libsts
    # links, so loading torch's makes libsts bind to it. Loaded the other way
    # round the process would hold two HIP runtimes and torch's would fail.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
    L.sts_required_bytes.argtypes = [u64, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.sts_init.argtypes = [ctypes.POINTER(vp), i32, u64, dbl, i32, vp, vp, ctypes.c_size_t, u64]
    L.sts_apply_gate.argtypes = [vp, i32, vp, vp]
    L.sts_truncate.argtypes = [vp]
    L.sts_peak.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(dbl)]
    L.sts_num_terms.argtypes = [vp, ctypes.POINTER(u64)]
    L.sts_read_terms.argtypes = [vp, u64, vp, vp, ctypes.POINTER(u64)]
    L.sts_load_terms.argtypes = [vp, u64, vp, vp]
    L.sts_stats.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(u64)]
    L.sts_counters.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.sts_profile.argtypes = [vp, i32]
    L.sts_kernel_time.argtypes = [vp, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(u64)]
    L.sts_free.argtypes = [vp]
    L.sts_free.restype = None
    L.sts_batch_run.argtypes = [i32, ctypes.POINTER(Circuit), ctypes.POINTER(BatchConfig),
                                ctypes.POINTER(CircuitResult)]
    L.sts_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ServerConfig)]
    L.sts_server_submit.argtypes = [vp, ctypes.POINTER(Circuit), ctypes.POINTER(u64)]
    L.sts_server_wait.argtypes = [vp, u64, ctypes.POINTER(CircuitResult)]
    L.sts_server_stats.argtypes = [vp] + [ctypes.POINTER(u64)] * 4
    L.sts_server_destroy.argtypes = [vp]
    L.sts_server_destroy.restype = None
    L.sts_set_sort_shape.argtypes = [vp, i32, i32]
    L.sts_step_static.argtypes = [i32, u64, dbl, i32, vp, i32, vp, vp, vp, vp, u64, vp, vp, vp, vp]
    L.sts_strerror.argtypes = [i32]
    L.sts_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("sts_free", "sts_strerror", "sts_server_destroy"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().sts_strerror(status).decode()


def _check(rc: int, what: str):
    if rc == STS_E_CAPACITY:
        raise CapacityError(rc, what)
    if rc != STS_OK:
        raise StsError(rc, what)


def step_static(n_qubits: int, K: int, p: float, precision, qubits: Sequence[int], U: np.ndarray,
                keys_in: int, amps_in: int, n_in: int, keys_out: int, amps_out: int, n_out: int,
                stats: int = 0, stream: int = 0) -> None:
    """sts_step_static: one gate step on device arrays given by address
    (keys u64, amplitudes complex128/complex64; n_out one u64, stats two
    doubles or 0), with no allocation; only enqueues work on the stream."""
    qs = (ctypes.c_int * len(qubits))(*[int(q) for q in qubits])
    u = np.ascontiguousarray(U, dtype=np.complex128)
    vp = ctypes.c_void_p
    _check(load().sts_step_static(int(n_qubits), int(K), float(p), _prec(precision), vp(stream or None), len(qubits),
                                  qs, u.ctypes.data_as(vp), vp(keys_in or None), vp(amps_in or None), int(n_in),
                                  vp(keys_out or None), vp(amps_out or None), vp(n_out or None), vp(stats or None)),
           "sts_step_static")


def required_bytes(cap_terms: int, precision: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().sts_required_bytes(int(cap_terms), int(precision), ctypes.byref(out)), "sts_required_bytes")
    return out.value


def _prec(precision) -> int:
    if precision in ("c128", STS_C128, "complex128"):
        return STS_C128
    if precision in ("c64", STS_C64, "complex64"):
        return STS_C64
    raise ValueError(f"precision {precision!r}")


class State:
    """A sparse, truncated state on one GPU.

    n:          qubits (1..64)
    K:          top-k limit (0 = off)
    p:          p-mass fraction (off unless 0 < p < 1)
    precision:  "c128" (FP64 amplitudes) or "c64" (FP32 amplitudes, FP64 masses)
    capacity:   most terms ever held (default max(K, 2^20))
    device:     CUDA/HIP device index; stream: a torch stream (default: current)
    """

    def __init__(self, n: int, K: int = 0, p: float = 0.0, precision="c128", capacity: Optional[int] = None,
                 device: int = 0, stream=None):
        import torch

        L = load()
        self.n = int(n)
        self.K = int(K)
        self.p = float(p)
        self.precision = _prec(precision)
        cap = int(capacity) if capacity else max(self.K, 1 << 20)
        self.capacity = cap
        self.device = torch.device("cuda", device)
        nbytes = required_bytes(cap, self.precision)
        # the arena: device memory owned by torch, carved by the library
        self._arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p(0)
        _check(L.sts_init(ctypes.byref(ctx), self.n, self.K, self.p, self.precision,
                          ctypes.c_void_p(self._stream.cuda_stream), ctypes.c_void_p(self._arena.data_ptr()),
                          nbytes, cap), "sts_init")
        self._ctx = ctx

    # -- core operations ------------------------------------------------
    def apply_gate(self, qubits: Sequence[int], U: np.ndarray):
        qs = np.ascontiguousarray(qubits, dtype=np.int32)
        u = np.ascontiguousarray(U, dtype=np.complex128)
        m = qs.shape[0]
        if u.shape != (1 << m, 1 << m):
            raise ValueError(f"U must be {1 << m}x{1 << m}")
        _check(load().sts_apply_gate(self._ctx, m, qs.ctypes.data, u.ctypes.data), "sts_apply_gate")

    def truncate(self):
        _check(load().sts_truncate(self._ctx), "sts_truncate")

    def peak(self) -> Tuple[int, float]:
        k = ctypes.c_uint64(0)
        pr = ctypes.c_double(0)
        _check(load().sts_peak(self._ctx, ctypes.byref(k), ctypes.byref(pr)), "sts_peak")
        return int(k.value), pr.value

    def num_terms(self) -> int:
        n = ctypes.c_uint64(0)
        _check(load().sts_num_terms(self._ctx, ctypes.byref(n)), "sts_num_terms")
        return int(n.value)

    def read_terms(self) -> Tuple[np.ndarray, np.ndarray]:
        """(keys uint64, amps complex128), ascending keys."""
        n = self.num_terms()
        keys = np.empty(max(n, 1), dtype=np.uint64)
        amps = np.empty(max(n, 1), dtype=np.complex128)
        got = ctypes.c_uint64(0)
        _check(load().sts_read_terms(self._ctx, n, keys.ctypes.data, amps.ctypes.data, ctypes.byref(got)),
               "sts_read_terms")
        return keys[: got.value].copy(), amps[: got.value].copy()

    def load_terms(self, keys: np.ndarray, amps: np.ndarray):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        a = np.ascontiguousarray(amps, dtype=np.complex128)
        if k.shape != a.shape:
            raise ValueError("keys and amps differ in length")
        _check(load().sts_load_terms(self._ctx, k.shape[0], k.ctypes.data, a.ctypes.data), "sts_load_terms")

    def set_sort_shape(self, small_log2: int, shape="8x16"):
        """Sort states of at most 2^small_log2 terms with `shape` ("8x16",
        "8x8", "11x16", "11x8": digit bits x keys per thread); 0 = default."""
        code = SORT_SHAPES[shape] if isinstance(shape, str) else int(shape)
        _check(load().sts_set_sort_shape(self._ctx, int(small_log2), code), "sts_set_sort_shape")

    def stats(self) -> dict:
        W, f, lc = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        c = ctypes.c_uint64(0)
        _check(load().sts_stats(self._ctx, ctypes.byref(W), ctypes.byref(f), ctypes.byref(lc), ctypes.byref(c)),
               "sts_stats")
        return dict(W=W.value, kept_fraction=f.value, log10_cum_kept=lc.value, candidates=int(c.value))

    def counters(self) -> dict:
        g, u, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(load().sts_counters(self._ctx, ctypes.byref(g), ctypes.byref(u), ctypes.byref(c)), "sts_counters")
        return dict(gate_steps=int(g.value), term_updates=int(u.value), candidates=int(c.value))

    def profile(self, enable: bool = True):
        _check(load().sts_profile(self._ctx, 1 if enable else 0), "sts_profile")

    def kernel_times(self, reset: bool = False) -> dict:
        """{kind: (total_ms, launches)} for every kernel kind."""
        out = {}
        L = load()
        for i, name in enumerate(KERNEL_KINDS):
            ms, n = ctypes.c_double(0), ctypes.c_uint64(0)
            last = reset and i == len(KERNEL_KINDS) - 1
            _check(L.sts_kernel_time(self._ctx, i, 1 if last else 0, ctypes.byref(ms), ctypes.byref(n)),
                   "sts_kernel_time")
            out[name] = (ms.value, int(n.value))
        return out

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load().sts_free(self._ctx)
            self._ctx = ctypes.c_void_p(0)
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
