"""A resident simulation server with continuous batching (sts_server_*).

    with Server(streams=8, max_active=4) as srv:
        t = srv.submit(circuit, K=1 << 16, p=0.99)
        result = srv.wait(t)

Requests are admitted in submission order whenever their context fits the
server's device memory budget; workers interleave their active requests a
few gates at a time. Every request computes exactly what it computes alone.
"""
from __future__ import annotations

import ctypes

from . import _lib
from .batch import _Packed


def _result(r) -> dict:
    return dict(status=r.status, peak_key=int(r.peak_key), peak_prob=r.peak_prob, n_terms=int(r.n_terms),
                gate_steps=int(r.gate_steps), term_updates=int(r.term_updates), log10_cum_kept=r.log10_cum_kept,
                seconds=r.seconds, queue_seconds=r.queue_seconds, latency_seconds=r.latency_seconds)


class Server:
    def __init__(self, precision="c64", streams: int = 8, max_active: int = 4, gates_per_turn: int = 8,
                 hbm_bytes: int = 0):
        L = _lib.load()
        cfg = _lib.ServerConfig(_lib._prec(precision), int(streams), int(max_active), int(gates_per_turn),
                                int(hbm_bytes))
        h = ctypes.c_void_p(0)
        _lib._check(L.sts_server_create(ctypes.byref(h), ctypes.byref(cfg)), "sts_server_create")
        self._h = h
        self._out = {}  # ticket -> packed circuit whose output arrays the server fills

    def submit(self, circuit, K: int = 0, p: float = 0.0, want_terms: bool = False) -> int:
        """Queue a request; with want_terms its result also holds the final
        'keys' and 'amps' (ascending keys)."""
        pk = _Packed(circuit, K, p, want_terms)  # the server copies the gate arrays before returning
        t = ctypes.c_uint64(0)
        _lib._check(_lib.load().sts_server_submit(self._h, ctypes.byref(pk.c), ctypes.byref(t)), "sts_server_submit")
        if want_terms:
            self._out[int(t.value)] = pk  # its output arrays must outlive the request
        return int(t.value)

    def wait(self, ticket: int) -> dict:
        r = _lib.CircuitResult()
        _lib._check(_lib.load().sts_server_wait(self._h, int(ticket), ctypes.byref(r)), "sts_server_wait")
        out = _result(r)
        pk = self._out.pop(int(ticket), None)
        if pk is not None:
            out["keys"], out["amps"] = pk.terms(out["n_terms"])
        return out

    def stats(self) -> dict:
        v = [ctypes.c_uint64(0) for _ in range(4)]
        _lib._check(_lib.load().sts_server_stats(self._h, *[ctypes.byref(x) for x in v]), "sts_server_stats")
        return dict(queued=v[0].value, active=v[1].value, done=v[2].value, bytes_in_use=v[3].value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().sts_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
