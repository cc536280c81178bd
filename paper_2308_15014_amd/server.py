"""Python surface of the serving loop (caps_server_* in include/caps.h):
argument marshalling only; scheduling, batching and search run in libcaps."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import SEARCH_DISJUNCTIVE, ServerParams, ServerStats, check, lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Server:
    """Continuous-batching server over one index (host-side requests)."""

    def __init__(self, index, *, k=10, nprobe=32, mode=0, routing=0, rerank=0, max_batch=4096, streams=2,
                 queue_slots=1 << 20, max_constraints=16, workspace_bytes=0, batch_window_us=0.0,
                 disjunctive=False):
        self.index = index          # keeps the index alive as long as the server
        self.k = k
        self.d = index.info()["d"]
        p = ServerParams(k, nprobe, mode, routing, rerank, max_batch, streams, queue_slots, max_constraints,
                         SEARCH_DISJUNCTIVE if disjunctive else 0, workspace_bytes, batch_window_us)
        h = ctypes.c_void_p()
        check(lib().caps_server_create(index._h, ctypes.byref(p), ctypes.byref(h)))
        self._h = h

    def submit(self, q, attrs=(), vals=()) -> int:
        q = np.ascontiguousarray(q, np.float32).reshape(-1)
        a = np.ascontiguousarray(attrs, np.int32)
        v = np.ascontiguousarray(vals, np.int32)
        t = ctypes.c_uint64()
        check(lib().caps_server_submit(self._h, _p(q), int(a.size), _p(a) if a.size else None,
                                       _p(v) if v.size else None, ctypes.byref(t)))
        return int(t.value)

    def replay(self, q, con_off, con_attr, con_val, arrival_s) -> np.ndarray:
        """Submits request i at arrival_s[i] seconds from now (blocking);
        returns the tickets (0 = refused by a full queue)."""
        q = np.ascontiguousarray(q, np.float32)
        co = np.ascontiguousarray(con_off, np.int32)
        ca = np.ascontiguousarray(con_attr, np.int32)
        cv = np.ascontiguousarray(con_val, np.int32)
        if ca.size == 0:
            ca = np.zeros(1, np.int32)
            cv = np.zeros(1, np.int32)
        ar = np.ascontiguousarray(arrival_s, np.float64)
        n = q.shape[0]
        tk = np.zeros(n, np.uint64)
        check(lib().caps_server_replay(self._h, _p(q), _p(co), _p(ca), _p(cv), n, _p(ar), _p(tk)))
        return tk

    def poll(self, max_results=65536) -> dict:
        tk = np.zeros(max_results, np.uint64)
        ids = np.zeros((max_results, self.k), np.int32)
        dist = np.zeros((max_results, self.k), np.float32)
        lat = np.zeros(max_results, np.float32)
        st = np.zeros(max_results, np.int32)
        n = ctypes.c_int32()
        check(lib().caps_server_poll(self._h, max_results, _p(tk), _p(ids), _p(dist), _p(lat), _p(st),
                                     ctypes.byref(n)))
        c = n.value
        return dict(tickets=tk[:c], ids=ids[:c], dist=dist[:c], latency_ms=lat[:c], status=st[:c])

    def drain(self, timeout_s=60.0):
        check(lib().caps_server_drain(self._h, timeout_s))

    def stats(self, reset=False) -> dict:
        s = ServerStats()
        check(lib().caps_server_stats(self._h, ctypes.byref(s), 1 if reset else 0))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_ if f != "reserved"}

    def close(self):
        if self._h:
            lib().caps_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
