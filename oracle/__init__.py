"""CPU oracle for CAPS filtered partitioned search (arXiv 2308.15014).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path never
imports, links or runs anything here, and nothing here imports the product.

`caps_oracle.c` holds the arithmetic (k-means, Attribute Frequency Tree,
CSR, routing, sub-partition choice, filter, distance, top-k, brute force);
this module only turns attributes into tokens and marshals arrays.

Token model (paper, Section 2 "Attribute Model"; Table 1 "Sparse
Attributes"): dense attribute i with value v is token off_i + v, where off
is the prefix sum of the dense vocabularies; label l is token off_L + l.  A
query constraint (attr, val) is the token of that pair; the filter of
Definition 1, with unconstrained attributes as wildcards, becomes "every
query token is held by the point".
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "caps_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MAX_LABELS = 8   # distinct label constraints a query may hold (more: answered as empty)


def build(force: bool = True) -> str:
    """Compile the oracle with strict FP semantics (no contraction, no
    fast-math) so each fmaf chain keeps its written order."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- tokens
@dataclasses.dataclass
class Tokens:
    tok_off: np.ndarray     # (N+1,) int64
    toks: np.ndarray        # (nnz,) int32
    tok_attr: np.ndarray    # (n_tok,) int32: dense attribute or -1 for labels
    n_tok: int
    dense_off: np.ndarray   # (L+1,) prefix sums of dense vocabularies
    n_dense: int
    label_vocab: int


def tokens_of(dense, dense_vocab, label_off, labels, label_vocab) -> Tokens:
    n_dense = 0 if dense is None else dense.shape[1]
    dense_off = np.zeros(n_dense + 1, dtype=np.int64)
    if n_dense:
        dense_off[1:] = np.cumsum(dense_vocab)
        if np.any(dense >= np.asarray(dense_vocab, dtype=np.uint32)[None, :]):
            raise ValueError("dense value outside its vocabulary")
    base = int(dense_off[-1])
    n = dense.shape[0] if dense is not None else len(label_off) - 1
    per = np.zeros(n, dtype=np.int64)
    if n_dense:
        per += n_dense
    if labels is not None:
        per += np.diff(label_off)
    tok_off = np.zeros(n + 1, dtype=np.int64)
    tok_off[1:] = np.cumsum(per)
    toks = np.zeros(int(tok_off[-1]), dtype=np.int32)
    if n_dense:
        idx = tok_off[:-1][:, None] + np.arange(n_dense)[None, :]
        toks[idx.ravel()] = (dense.astype(np.int64) + dense_off[:-1][None, :]).ravel()
    if labels is not None:
        start = tok_off[:-1] + n_dense
        cnt = np.diff(label_off)
        owner = np.repeat(np.arange(n), cnt)
        rank = np.arange(len(labels)) - np.repeat(label_off[:-1], cnt)
        if len(labels) and int(labels.max()) >= label_vocab:
            raise ValueError("label outside its vocabulary")
        toks[start[owner] + rank] = base + labels.astype(np.int64)
    n_tok = base + (label_vocab if labels is not None else 0)
    tok_attr = np.full(n_tok, -1, dtype=np.int32)
    for a in range(n_dense):
        tok_attr[dense_off[a]:dense_off[a + 1]] = a
    return Tokens(tok_off, toks, tok_attr, n_tok, dense_off, n_dense,
                  label_vocab if labels is not None else 0)


def query_tokens(tk: Tokens, con_off, con_attr, con_val, disjunctive: bool = False):
    """Constraint pairs -> token CSR plus a per-query flag for pairs whose
    attribute or value lies outside the index's vocabularies.

    disjunctive=True (Section 5.3: several attributes joined with OR): a pair
    with attr == -1 separates AND-terms and becomes token -1; a pair outside
    the vocabularies makes only its own term unsatisfiable (token -2 in that
    term), and so does a term asking for more than MAX_LABELS labels."""
    con_off = np.asarray(con_off, dtype=np.int64)
    a = np.asarray(con_attr, dtype=np.int64)
    v = np.asarray(con_val, dtype=np.int64)
    nq = len(con_off) - 1
    tok = np.zeros(len(a), dtype=np.int64)
    bad_pair = np.zeros(len(a), dtype=bool)
    is_dense = (a >= 0) & (a < tk.n_dense)
    if tk.n_dense:
        voc = np.diff(tk.dense_off)
        ad = np.where(is_dense, a, 0)
        ok = is_dense & (v >= 0) & (v < voc[ad])
        tok = np.where(ok, tk.dense_off[ad] + v, tok)
        bad_pair |= is_dense & ~ok
    is_lab = a == tk.n_dense
    if tk.label_vocab:
        ok = is_lab & (v >= 0) & (v < tk.label_vocab)
        tok = np.where(ok, tk.dense_off[-1] + v, tok)
        bad_pair |= is_lab & ~ok
    else:
        bad_pair |= is_lab
    bad_pair |= (a < 0) | (a > tk.n_dense)
    q_bad = np.zeros(nq, dtype=np.uint8)
    if disjunctive:
        sep = a == -1
        tok = np.where(sep, -1, np.where(bad_pair, -2, tok))
        # a term asking for more than MAX_LABELS distinct labels is outside
        # the build's limits: unsatisfiable
        for qi in range(nq):
            lo, hi = int(con_off[qi]), int(con_off[qi + 1])
            start = lo
            for e in range(lo, hi + 1):
                if e < hi and not sep[e]:
                    continue
                if len(set(v[start:e][is_lab[start:e]].tolist())) > MAX_LABELS:
                    tok[start:e] = -2
                start = e + 1
        return con_off.astype(np.int64), tok.astype(np.int32), q_bad
    tok = np.where(bad_pair, 0, tok)
    owner = np.repeat(np.arange(nq), np.diff(con_off))
    if len(a):
        np.maximum.at(q_bad, owner, bad_pair.astype(np.uint8))
    # a query asking for more than MAX_LABELS distinct labels is outside the
    # build's limits and answered as empty (it chooses no sub-partition)
    for qi in range(nq):
        lo, hi = con_off[qi], con_off[qi + 1]
        if len(set(v[lo:hi][is_lab[lo:hi]].tolist())) > MAX_LABELS:
            q_bad[qi] = 1
    return con_off.astype(np.int64), tok.astype(np.int32), q_bad


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's parallel loops (n <= 0: unchanged); returns
    the count in effect."""
    L = lib()
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = ctypes.c_int
    return int(L.orc_set_threads(int(n)))


# ---------------------------------------------------------------- sampler
def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    lib().orc_splitmix64_first.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p]
    lib().orc_splitmix64_first.restype = ctypes.c_uint64
    lib().orc_splitmix64_first(ctypes.c_uint64(seed & (2**64 - 1)), count, _p(out))
    return out


def init_ids(seed: int, n: int, b: int) -> np.ndarray:
    out = np.zeros(b, dtype=np.int32)
    L = lib()
    L.orc_init_ids.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
    rc = L.orc_init_ids(ctypes.c_uint64(seed & (2**64 - 1)), n, b, _p(out))
    if rc != 0:
        raise ValueError("init_ids: b must be in [0, n]")
    return out


# ---------------------------------------------------------------- k-means
def assign(x, cent, metric=0) -> np.ndarray:
    x = _c(x, np.float32)
    cent = _c(cent, np.float32)
    out = np.zeros(x.shape[0], dtype=np.int32)
    L = lib()
    L.orc_assign.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                             ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_assign(_p(x), x.shape[0], x.shape[1], _p(cent), cent.shape[0], metric, _p(out))
    return out


def update(x, a, cent, metric=0) -> np.ndarray:
    x = _c(x, np.float32)
    c = _c(cent, np.float32).copy()
    a = _c(a, np.int32)
    L = lib()
    L.orc_update.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                             ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_update(_p(x), x.shape[0], x.shape[1], _p(a), c.shape[0], metric, _p(c))
    return c


def centroid_norms(cent) -> np.ndarray:
    cent = _c(cent, np.float32)
    out = np.zeros(cent.shape[0], dtype=np.float32)
    L = lib()
    L.orc_centroid_norms.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.orc_centroid_norms(_p(cent), cent.shape[0], cent.shape[1], _p(out))
    return out


def kmeans(x, b, iters, metric=0, init=None, seed=0):
    x = _c(x, np.float32)
    n, d = x.shape
    if init is None:
        init = init_ids(seed, n, b)
    init = _c(init, np.int32)
    cent = np.zeros((b, d), dtype=np.float32)
    a = np.zeros(n, dtype=np.int32)
    L = lib()
    L.orc_kmeans.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p]
    L.orc_kmeans(_p(x), n, d, b, iters, metric, _p(init), _p(cent), _p(a))
    return cent, a


def objective(x, cent, a) -> float:
    x = _c(x, np.float32)
    L = lib()
    L.orc_objective.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p]
    L.orc_objective.restype = ctypes.c_double
    return float(L.orc_objective(_p(x), x.shape[0], x.shape[1], _p(_c(cent, np.float32)),
                                 _p(_c(a, np.int32))))


# ---------------------------------------------------------------- AFT + CSR
def aft(a, b, h, tk: Tokens):
    a = _c(a, np.int32)
    n = a.shape[0]
    tags = np.zeros(b * h, dtype=np.int32)
    level = np.zeros(n, dtype=np.int8)
    L = lib()
    L.orc_aft.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                          ctypes.c_void_p]
    rc = L.orc_aft(n, _p(a), b, h, _p(tk.tok_off), _p(tk.toks), tk.n_tok, _p(tags), _p(level))
    if rc != 0:
        raise MemoryError("orc_aft")
    return tags.reshape(b, h), level


def attribute_order(dense, n):
    """The ids sorted by their dense attribute values, attribute 0 first,
    ties by ascending id (a stable lexicographic sort); ascending ids when
    there are no dense attributes."""
    if dense is None or np.asarray(dense).size == 0:
        return np.arange(n, dtype=np.int32)
    dense = np.asarray(dense)
    return np.lexsort(tuple(dense[:, j] for j in range(dense.shape[1] - 1, -1, -1))).astype(np.int32)


def csr(a, level, b, h, dense=None, order=None):
    """CSR layout (Appendix "Index size"): points grouped by (partition,
    level); inside a sub-partition in `order` (default: attribute_order of
    `dense`, i.e. by dense attribute values, then id)."""
    a = _c(a, np.int32)
    level = _c(level, np.int8)
    n = a.shape[0]
    if order is None:
        order = attribute_order(dense, n)
    order = _c(order, np.int32)
    assert order.shape == (n,)
    perm = np.zeros(n, dtype=np.int32)
    offs = np.zeros(b * (h + 1) + 1, dtype=np.int32)
    L = lib()
    L.orc_csr.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_csr(n, _p(a), _p(level), b, h, _p(order), _p(perm), _p(offs))
    return perm, offs


@dataclasses.dataclass
class Index:
    x: np.ndarray
    tk: Tokens
    metric: int
    b: int
    h: int
    centroids: np.ndarray
    assign: np.ndarray
    tags: np.ndarray      # (b, h)
    level: np.ndarray
    perm: np.ndarray
    offs: np.ndarray
    init: np.ndarray


def build_index(x, dense, dense_vocab, label_off, labels, label_vocab, *, metric, b, h,
                iters, seed, init=None) -> Index:
    """Algorithm 1: f = seeded Lloyd k-means, then the truncated AFT in every
    partition, then the CSR layout."""
    x = _c(x, np.float32)
    tk = tokens_of(dense, dense_vocab, label_off, labels, label_vocab)
    if init is None:
        init = init_ids(seed, x.shape[0], b)
    cent, a = kmeans(x, b, iters, metric, init=init)
    tags, level = aft(a, b, h, tk)
    perm, offs = csr(a, level, b, h, dense)
    return Index(x, tk, metric, b, h, cent, a, tags, level, perm, offs, np.asarray(init))


def bliss_assign(cand, b) -> np.ndarray:
    """Section 5.2 (CAPS-BLISS) re-partitioning: every item in ascending id to
    the least loaded of its K candidate buckets (best first), ties to the
    better-ranked one."""
    cand = _c(cand, np.int32)
    n, k = cand.shape
    out = np.zeros(n, dtype=np.int32)
    L = lib()
    L.orc_bliss_assign.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p]
    if L.orc_bliss_assign(_p(cand), n, k, int(b), _p(out)) != 0:
        raise ValueError("candidate outside [0, b)")
    return out


def build_assigned(x, dense, dense_vocab, label_off, labels, label_vocab, assign, *, metric, b, h,
                   seed, init=None) -> Index:
    """Algorithm 1 with given first-level partitions (learned partitions,
    Section 5.2): each centroid is one Lloyd update of the sampled initial
    centroids with the given assignment (the mean of its points; an empty
    partition keeps its initial point), then the truncated AFT and the CSR."""
    x = _c(x, np.float32)
    tk = tokens_of(dense, dense_vocab, label_off, labels, label_vocab)
    if init is None:
        init = init_ids(seed, x.shape[0], b)
    a = _c(assign, np.int32)
    cent = update(x, a, x[np.asarray(init)], metric)
    tags, level = aft(a, b, h, tk)
    perm, offs = csr(a, level, b, h, dense)
    return Index(x, tk, metric, b, h, cent, a, tags, level, perm, offs, np.asarray(init))


def insert(idx: Index, x_new, dense_new, label_off_new, labels_new) -> Index:
    """Dynamic insertion (Table 1; Section 1 "Practical Utility"): the new
    points get ids n, n+1, ... and join the frozen partition model -- the
    centroid the k-means assignment picks, then the first tagged level whose
    tag they hold, else the remainder; centroids and tags are unchanged and
    the CSR is laid out again: the points already present in their order,
    each new point at the end of its sub-partition, in ascending id."""
    x_new = _c(x_new, np.float32)
    n_new = x_new.shape[0]
    tk = idx.tk
    dense_vocab = np.diff(tk.dense_off).astype(np.int64)
    tkn = tokens_of(dense_new, dense_vocab, label_off_new, labels_new, tk.label_vocab)
    if tkn.n_tok != tk.n_tok:
        raise ValueError("new points must carry the index's attribute kinds")
    a_new = assign(x_new, idx.centroids, idx.metric)
    lev_new = np.zeros(n_new, dtype=np.int8)
    L = lib()
    L.orc_insert_levels.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    tags = _c(idx.tags.reshape(-1), np.int32) if idx.h > 0 else np.zeros(1, np.int32)
    L.orc_insert_levels(n_new, _p(a_new), _p(tags), idx.h, _p(tkn.tok_off), _p(tkn.toks), _p(lev_new))
    tok_off = np.concatenate([tk.tok_off, tk.tok_off[-1] + tkn.tok_off[1:]])
    allt = Tokens(tok_off, np.concatenate([tk.toks, tkn.toks]), tk.tok_attr, tk.n_tok, tk.dense_off, tk.n_dense,
                  tk.label_vocab)
    a_all = np.concatenate([idx.assign, a_new]).astype(np.int32)
    l_all = np.concatenate([idx.level, lev_new]).astype(np.int8)
    # the points already present keep their CSR order; the new ones follow
    # at the end of their sub-partition in ascending id
    perm, offs = csr(a_all, l_all, idx.b, idx.h,
                     order=np.concatenate([idx.perm, np.arange(idx.x.shape[0], idx.x.shape[0] + n_new)]))
    return Index(np.concatenate([idx.x, x_new]), allt, idx.metric, idx.b, idx.h, idx.centroids, a_all,
                 idx.tags, l_all, perm, offs, idx.init)


def build_from_workload(w, **over) -> Index:
    kw = dict(metric=w.metric, b=w.n_partitions, h=w.aft_height, iters=w.kmeans_iters,
              seed=w.seed)
    kw.update(over)
    return build_index(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, **kw)


# ---------------------------------------------------------------- queries
@dataclasses.dataclass
class Result:
    ids: np.ndarray
    dist: np.ndarray
    n_cand: np.ndarray
    n_surv: np.ndarray
    probes: Optional[np.ndarray] = None
    masks: Optional[np.ndarray] = None


def search(idx: Index, q, con_off, con_attr, con_val, k, m, rule=0, disjunctive=False) -> Result:
    """Algorithm 2 over a query batch (rule 0: exact sub-partition choice;
    rule 1: the algorithm's one-sub-partition choice read literally).
    disjunctive=True: constraint lists are OR-ed AND-terms separated by
    attr == -1 (the chosen sub-partitions are the union over the terms)."""
    q = _c(q, np.float32)
    nq, d = q.shape
    qo, qt, qbad = query_tokens(idx.tk, con_off, con_attr, con_val, disjunctive)
    ids = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float32)
    nc = np.zeros(nq, dtype=np.int64)
    ns = np.zeros(nq, dtype=np.int64)
    probes = np.zeros((nq, m), dtype=np.int32)
    masks = np.zeros((nq, m), dtype=np.uint32)
    tags = _c(idx.tags.reshape(-1), np.int32)
    L = lib()
    vp = ctypes.c_void_p
    L.orc_search.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32,
                             ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp,
                             vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                             vp, vp, vp]
    rc = L.orc_search(_p(idx.x), idx.x.shape[0], d, _p(idx.tk.tok_off), _p(idx.tk.toks),
                      _p(idx.tk.tok_attr), _p(_c(idx.centroids, np.float32)), idx.b, idx.metric,
                      _p(tags), idx.h, _p(idx.perm), _p(idx.offs), _p(q), nq, _p(qo), _p(qt),
                      _p(qbad), k, m, rule, _p(ids), _p(dist), _p(nc), _p(ns), _p(probes),
                      _p(masks))
    if rc != 0:
        raise ValueError("orc_search: bad k or m")
    return Result(ids, dist, nc, ns, probes, masks)


def bruteforce(x, tk: Tokens, metric, q, con_off, con_attr, con_val, k, disjunctive=False) -> Result:
    """Exact filtered top-k in FP32 (Appendix "Groundtruth")."""
    x = _c(x, np.float32)
    q = _c(q, np.float32)
    nq, d = q.shape
    qo, qt, qbad = query_tokens(tk, con_off, con_attr, con_val, disjunctive)
    ids = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float32)
    nv = np.zeros(nq, dtype=np.int64)
    L = lib()
    vp = ctypes.c_void_p
    L.orc_bruteforce.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, ctypes.c_int32,
                                 vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    L.orc_bruteforce(_p(x), x.shape[0], d, _p(tk.tok_off), _p(tk.toks), _p(tk.tok_attr), metric,
                     _p(q), nq, _p(qo), _p(qt), _p(qbad), k, _p(ids), _p(dist), _p(nv))
    return Result(ids, dist, nv, nv)


def workload_tokens(w) -> Tokens:
    return tokens_of(w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab)
