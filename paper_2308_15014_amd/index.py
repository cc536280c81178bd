"""Python surface over libcaps: argument marshalling only.

Device memory and streams come from PyTorch; every step of build and search
runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from ._lib import (PREC, SEARCH_DISJUNCTIVE, SEARCH_VALIDATE, BuildParams, IndexInfo, RouterInfo, RouterParams,
                   SearchParams, check, lib)


def _torch():
    import torch
    return torch


def _host(a, dtype):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dev(t, dtype, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Index:
    """A CAPS index resident on one GPU."""

    def __init__(self, handle: ctypes.c_void_p, device):
        self._h = handle
        self.device = device
        self._info = None

    # ------------------------------------------------------------ build
    @classmethod
    def build(cls, x, dense=None, dense_vocab=None, label_off=None, labels=None, label_vocab=0, *,
              metric: int = 0, n_partitions: int, kmeans_iters: int = 10, aft_height: int = 2,
              seed: int = 0, init_ids=None, precision="none", assign=None, device=None,
              stream=None) -> "Index":
        """Algorithm 1 on the current (or given) device.  `assign` (n
        partition ids, e.g. from bliss_assign) replaces the k-means
        partitions with given ones."""
        torch = _torch()
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        x = _host(x, np.float32)
        n, d = x.shape
        dense = _host(dense, np.uint32)
        n_dense = 0 if dense is None else dense.shape[1]
        vocab = _host(dense_vocab, np.int32) if n_dense else None
        lo = _host(label_off, np.int64)
        lb = _host(labels, np.uint32)
        if lb is not None and lb.size == 0:
            lb = np.zeros(1, dtype=np.uint32)
        init = _host(init_ids, np.int32)
        asg = _host(assign, np.int32)
        if asg is not None and asg.shape != (n,):
            raise ValueError("assign must hold one partition per point")
        prec = PREC[precision] if isinstance(precision, str) else int(precision)
        p = BuildParams(metric, n_partitions, kmeans_iters, aft_height,
                        ctypes.c_uint64(seed & (2**64 - 1)).value, _ptr(init), prec, 0, _ptr(asg))
        out = ctypes.c_void_p()
        with torch.cuda.device(device):
            st = _stream(stream)
            check(lib().caps_build(_ptr(x), n, d, _ptr(dense), n_dense, _ptr(vocab), _ptr(lo),
                                   _ptr(lb), int(label_vocab) if lo is not None else 0,
                                   ctypes.byref(p), st, ctypes.byref(out)))
        return cls(out, device)

    @classmethod
    def from_workload(cls, w, **over) -> "Index":
        kw = dict(metric=w.metric, n_partitions=w.n_partitions, kmeans_iters=w.kmeans_iters,
                  aft_height=w.aft_height, seed=w.seed)
        kw.update(over)
        return cls.build(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, **kw)

    def insert(self, x, dense=None, label_off=None, labels=None, stream=None):
        """Dynamic insertion of new points (ids continue after the existing
        ones); host arrays as for build."""
        torch = _torch()
        x = _host(x, np.float32)
        dense = _host(dense, np.uint32)
        lo = _host(label_off, np.int64)
        lb = _host(labels, np.uint32)
        if lb is not None and lb.size == 0:
            lb = np.zeros(1, dtype=np.uint32)
        with torch.cuda.device(self.device):
            check(lib().caps_insert(self._h, _ptr(x), int(x.shape[0]), _ptr(dense), _ptr(lo), _ptr(lb),
                                    _stream(stream)))
        self._info = None

    def save(self, path: str):
        check(lib().caps_save(self._h, str(path).encode()))

    @classmethod
    def load(cls, path: str, device=None) -> "Index":
        torch = _torch()
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        out = ctypes.c_void_p()
        with torch.cuda.device(device):
            check(lib().caps_load(str(path).encode(), None, ctypes.byref(out)))
        return cls(out, device)

    # ------------------------------------------------------------ query
    def _qargs(self, q, con_off, con_attr, con_val):
        torch = _torch()
        qd = _dev(q, torch.float32, self.device)
        co = _dev(con_off, torch.int32, self.device)
        ca = _dev(con_attr, torch.int32, self.device)
        cv = _dev(con_val, torch.int32, self.device)
        if ca.numel() == 0:
            ca = torch.zeros(1, dtype=torch.int32, device=self.device)
            cv = torch.zeros(1, dtype=torch.int32, device=self.device)
            n_con = 0
        else:
            n_con = int(ca.numel())
        return qd, co, ca, cv, n_con

    def search(self, q, con_off, con_attr, con_val, k: int, nprobe: int, *, rule: int = 0,
               mode: int = 0, rerank: int = 0, routing: int = 0, stream=None, counters: bool = False,
               out=None, workspace_bytes: int = 0, validate: bool = False, disjunctive: bool = False,
               rescue_grid: int = 0):
        """Top-k filtered search for a batch.  Returns device tensors
        (ids int32 [Q,k], dist float32 [Q,k]) and, with counters=True, the
        per-query candidate and survivor counts.  mode 1 scans the
        low-precision copy with matrix cores and rescores `rerank`
        candidates per query exactly; mode 2 forces the plain FP32 scan.
        routing 1 uses the learned router (with its centroid fallback).
        workspace_bytes caps the device workspace of the call (0: 4 GiB);
        the batch is searched in sub-batches that fit it.  validate=True
        synchronises and raises on NaN/Inf query rows; disjunctive=True lets
        a constraint pair with attr == OR (-1) separate AND-terms."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        nq = int(qd.shape[0])
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=self.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        else:
            ids, dist = out
        nc = torch.empty(nq, dtype=torch.int32, device=self.device) if counters else None
        ns = torch.empty(nq, dtype=torch.int32, device=self.device) if counters else None
        sp = self._sparams(k, nprobe, rule, mode, rerank, routing, workspace_bytes, validate, disjunctive,
                           rescue_grid)
        with torch.cuda.device(self.device):
            st = _stream(stream)
            check(lib().caps_search(self._h, ctypes.byref(sp), qd.data_ptr(), nq, co.data_ptr(),
                                    ca.data_ptr(), cv.data_ptr(), n_con, ids.data_ptr(),
                                    dist.data_ptr(), nc.data_ptr() if counters else None,
                                    ns.data_ptr() if counters else None, st))
        if counters:
            return ids, dist, nc, ns
        return ids, dist

    def search_static(self, q, con_off, con_attr, con_val, k: int, nprobe: int, *, rule: int = 0, mode: int = 0,
                      rerank: int = 0, routing: int = 0, stream=None, counters: bool = False, out=None,
                      workspace_bytes: int = 0, disjunctive: bool = False):
        """caps_search_static: the same search in the library's static device
        workspace (no allocation by the library; outputs allocated here unless
        `out` = (ids, dist) is given)."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        nq = int(qd.shape[0])
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=self.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        else:
            ids, dist = out
        nc = torch.empty(nq, dtype=torch.int32, device=self.device) if counters else None
        ns = torch.empty(nq, dtype=torch.int32, device=self.device) if counters else None
        sp = self._sparams(k, nprobe, rule, mode, rerank, routing, workspace_bytes, False, disjunctive)
        with torch.cuda.device(self.device):
            check(lib().caps_search_static(self._h, ctypes.byref(sp), qd.data_ptr(), nq, co.data_ptr(),
                                           ca.data_ptr(), cv.data_ptr(), n_con, ids.data_ptr(), dist.data_ptr(),
                                           nc.data_ptr() if counters else None, ns.data_ptr() if counters else None,
                                           _stream(stream)))
        if counters:
            return ids, dist, nc, ns
        return ids, dist

    @staticmethod
    def _sparams(k, nprobe, rule=0, mode=0, rerank=0, routing=0, workspace_bytes=0, validate=False,
                 disjunctive=False, rescue_grid=0):
        flags = (SEARCH_VALIDATE if validate else 0) | (SEARCH_DISJUNCTIVE if disjunctive else 0)
        return SearchParams(k, nprobe, rule, mode, rerank, routing, flags, rescue_grid, workspace_bytes)

    def workspace_bytes(self, n_q: int, k: int, nprobe: int, *, mode: int = 0, rerank: int = 0,
                        routing: int = 0, workspace_bytes: int = 0) -> int:
        """Device bytes one search call of n_q queries allocates."""
        sp = self._sparams(k, nprobe, 0, mode, rerank, routing, workspace_bytes)
        out = ctypes.c_int64()
        check(lib().caps_search_workspace(self._h, ctypes.byref(sp), n_q, ctypes.byref(out)))
        return int(out.value)

    def search_debug(self, q, con_off, con_attr, con_val, k: int, nprobe: int, *, rule: int = 0,
                     mode: int = 0, rerank: int = 0, routing: int = 0, disjunctive: bool = False,
                     rescue_grid: int = 0, workspace_bytes: int = 0):
        """caps_search_debug: (ids, dist, ncand, nsurv, surv_mask) with surv_mask
        [Q, ceil(n/64)] int64 words of filter pass bits over CSR positions."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        nq = int(qd.shape[0])
        words = (self.info()["n"] + 63) // 64
        ids = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        nc = torch.empty(nq, dtype=torch.int32, device=self.device)
        ns = torch.empty(nq, dtype=torch.int32, device=self.device)
        mask = torch.empty((nq, words), dtype=torch.int64, device=self.device)
        sp = self._sparams(k, nprobe, rule, mode, rerank, routing, workspace_bytes, False, disjunctive, rescue_grid)
        with torch.cuda.device(self.device):
            check(lib().caps_search_debug(self._h, ctypes.byref(sp), qd.data_ptr(), nq, co.data_ptr(),
                                          ca.data_ptr(), cv.data_ptr(), n_con, ids.data_ptr(), dist.data_ptr(),
                                          nc.data_ptr(), ns.data_ptr(), mask.data_ptr(), _stream(None)))
        return ids, dist, nc, ns, mask

    def probes(self, q, con_off, con_attr, con_val, nprobe: int, *, rule: int = 0, routing: int = 0,
               k: int = 1, stream=None, disjunctive: bool = False, mode: int = 0):
        """Routing and sub-partition choice only: (probes [Q,m], masks [Q,m])."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        nq = int(qd.shape[0])
        pr = torch.empty((nq, nprobe), dtype=torch.int32, device=self.device)
        mk = torch.empty((nq, nprobe), dtype=torch.int32, device=self.device)
        sp = self._sparams(k, nprobe, rule, mode, 0, routing, disjunctive=disjunctive)
        with torch.cuda.device(self.device):
            st = _stream(stream)
            check(lib().caps_search_probes(self._h, ctypes.byref(sp), qd.data_ptr(), nq, co.data_ptr(),
                                           ca.data_ptr(), cv.data_ptr(), n_con, pr.data_ptr(),
                                           mk.data_ptr(), st))
        return pr, mk

    # ------------------------------------------------------------ learned router
    @staticmethod
    def _rparams(hidden=1024, epochs=1, batch=4096, reset=1, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 in_scale=1.0, in_shift=0.0, fallback_prob=0.0, seed=0):
        return RouterParams(hidden, epochs, batch, reset, lr, beta1, beta2, eps, in_scale, in_shift,
                            fallback_prob, 0, ctypes.c_uint64(seed & (2**64 - 1)).value)

    def router_labels(self, ids):
        """Distinct partitions of each row of `ids` (device int32 n x k), -1 padded."""
        torch = _torch()
        ids = _dev(ids, torch.int32, self.device)
        n, k = ids.shape
        out = torch.empty((n, k), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            check(lib().caps_router_labels(self._h, ids.data_ptr(), n, k, out.data_ptr(), _stream(None)))
        return out

    def router_train(self, q, con_off, con_attr, con_val, labels, **params):
        """Trains the learned router on the GPU; returns the mean loss per epoch."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        lb = _dev(labels, torch.int32, self.device)
        p = self._rparams(**params)
        loss = np.zeros(max(p.epochs, 1), np.float32)
        with torch.cuda.device(self.device):
            check(lib().caps_router_train(self._h, ctypes.byref(p), qd.data_ptr(), int(qd.shape[0]),
                                          co.data_ptr(), ca.data_ptr(), cv.data_ptr(), n_con, lb.data_ptr(),
                                          int(lb.shape[1]), _ptr(loss), _stream(None)))
        return loss[:p.epochs]

    def router_set(self, w1=None, b1=None, w2=None, b2=None, **params):
        p = self._rparams(**params)
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (w1, b1, w2, b2)]
        check(lib().caps_router_set(self._h, ctypes.byref(p), *(_ptr(a) for a in arrs)))

    def router_info(self) -> dict:
        inf = RouterInfo()
        check(lib().caps_router_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in RouterInfo._fields_}

    def router_get(self) -> dict:
        inf = self.router_info()
        h, dp, b = inf["hidden"], inf["dpad"], inf["n_out"]
        out = dict(w1=np.zeros((h, dp), np.float32), b1=np.zeros(h, np.float32),
                   w2=np.zeros((b, h), np.float32), b2=np.zeros(b, np.float32))
        check(lib().caps_router_get(self._h, *(_ptr(out[k]) for k in ("w1", "b1", "w2", "b2"))))
        return out

    def router_logits(self, q, con_off, con_attr, con_val):
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        n = int(qd.shape[0])
        out = torch.empty((n, self.info()["n_partitions"]), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            check(lib().caps_router_logits(self._h, qd.data_ptr(), n, co.data_ptr(), ca.data_ptr(),
                                           cv.data_ptr(), n_con, out.data_ptr(), _stream(None)))
        return out

    def router_grads(self, q, con_off, con_attr, con_val, labels):
        """(loss, {w1, b1, w2, b2} gradients) of one batch, no update."""
        torch = _torch()
        qd, co, ca, cv, n_con = self._qargs(q, con_off, con_attr, con_val)
        lb = _dev(labels, torch.int32, self.device)
        g = {k: np.zeros_like(v) for k, v in self.router_get().items()}
        loss = np.zeros(1, np.float32)
        with torch.cuda.device(self.device):
            check(lib().caps_router_grads(self._h, qd.data_ptr(), int(qd.shape[0]), co.data_ptr(),
                                          ca.data_ptr(), cv.data_ptr(), n_con, lb.data_ptr(), int(lb.shape[1]),
                                          _ptr(loss), *(_ptr(g[k]) for k in ("w1", "b1", "w2", "b2")),
                                          _stream(None)))
        return float(loss[0]), g

    # ------------------------------------------------------------ inspection
    def info(self) -> dict:
        inf = IndexInfo()
        check(lib().caps_index_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in IndexInfo._fields_}

    def export(self) -> dict:
        inf = self.info()
        n, d, b, h = inf["n"], inf["d"], inf["n_partitions"], inf["aft_height"]
        out = dict(centroids=np.zeros((b, d), np.float32), assign=np.zeros(n, np.int32),
                   level=np.zeros(n, np.int8), perm=np.zeros(n, np.int32),
                   offs=np.zeros(b * (h + 1) + 1, np.int32), tags=np.zeros((b, max(h, 1)), np.int32))
        check(lib().caps_index_export(self._h, *(_ptr(out[k]) for k in
                                                 ("centroids", "assign", "level", "perm", "offs",
                                                  "tags"))))
        out["tags"] = out["tags"][:, :h]
        return out

    def export_lowp(self) -> dict:
        """Low-precision copy: codes [n, dpad] (uint16 bit patterns or uint8
        FP8 codes), per-vector scales (FP8) and exact |x|^2, CSR order."""
        inf = self.info()
        n, prec, dpad = inf["n"], inf["precision"], inf["lowp_dpad"]
        codes = np.zeros((n, dpad), np.uint8 if prec == PREC["fp8"] else np.uint16)
        scale = np.zeros(n, np.float32)
        xnorm = np.zeros(n, np.float32)
        check(lib().caps_index_export_lowp(self._h, _ptr(codes), _ptr(scale), _ptr(xnorm)))
        return dict(codes=codes, scale=scale, xnorm=xnorm, precision=prec)

    def close(self):
        if self._h:
            lib().caps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bliss_assign(cand, n_partitions: int) -> np.ndarray:
    """Re-partitioning of learned partitions (caps_bliss_assign): each point,
    in ascending id, to the least loaded of its candidate partitions (n x K,
    best first), ties to the earlier one.  Host arrays in and out."""
    cand = np.ascontiguousarray(np.asarray(cand), dtype=np.int32)
    if cand.ndim != 2:
        raise ValueError("cand must be n x K")
    n, k = cand.shape
    out = np.zeros(n, dtype=np.int32)
    check(lib().caps_bliss_assign(_ptr(cand), n, k, int(n_partitions), _ptr(out)))
    return out

