"""FP64 filtered brute force and recall (TEST INFRASTRUCTURE ONLY).

Appendix "Groundtruth": the true constrained neighbours are found by an
exact search over the valid points.  Here validity is evaluated directly on
the raw attribute arrays (Definition 1, unconstrained attributes as
wildcards) and distances in float64, independent of the C oracle's token
machinery and FP32 arithmetic.  Appendix "Metric": RecallK@K is
|index-topK intersect true-topK| / K.
"""
from __future__ import annotations

import numpy as np


def valid_mask(dense, label_off, labels, pairs, n_dense, dense_vocab=None, label_vocab=0):
    """Boolean mask of points satisfying every (attr, val) pair."""
    n = dense.shape[0] if dense is not None else len(label_off) - 1
    m = np.ones(n, dtype=bool)
    for a, v in pairs:
        if a < 0 or a > n_dense:
            return np.zeros(n, dtype=bool)
        if a < n_dense:
            if v < 0 or (dense_vocab is not None and v >= dense_vocab[a]):
                return np.zeros(n, dtype=bool)
            m &= dense[:, a] == v
        else:
            if labels is None or v < 0 or v >= label_vocab:
                return np.zeros(n, dtype=bool)
            has = np.zeros(n, dtype=bool)
            owner = np.repeat(np.arange(n), np.diff(label_off))
            has[owner[labels == v]] = True
            m &= has
    return m


def valid_mask_dnf(dense, label_off, labels, pairs, n_dense, dense_vocab=None, label_vocab=0, max_terms=4):
    """Points satisfying at least one AND-term of a disjunction whose terms
    are separated by pairs with attr == -1 (OR); more than max_terms terms
    make the query unsatisfiable (the build's limit)."""
    n = dense.shape[0] if dense is not None else len(label_off) - 1
    terms, cur = [], []
    for a, v in pairs:
        if a == -1:
            terms.append(cur)
            cur = []
        else:
            cur.append((a, v))
    terms.append(cur)
    m = np.zeros(n, dtype=bool)
    if len(terms) > max_terms:
        return m
    for t in terms:
        m |= valid_mask(dense, label_off, labels, t, n_dense, dense_vocab, label_vocab)
    return m


def pairs_of(con_off, con_attr, con_val, qi):
    lo, hi = int(con_off[qi]), int(con_off[qi + 1])
    return [(int(con_attr[e]), int(con_val[e])) for e in range(lo, hi)]


def dist64(x, q, metric):
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if metric == 0:
        t = x - q[None, :]
        return np.einsum("ij,ij->i", t, t)
    return x @ q


def topk64(x, dense, label_off, labels, dense_vocab, label_vocab, metric, q, con_off,
           con_attr, con_val, k, queries=None, disjunctive=False):
    """Per query: (ids, dists) of the exact filtered top-k in FP64, ties
    broken by the smaller id, padded with -1.  Also returns |D_C|."""
    n_dense = 0 if dense is None else dense.shape[1]
    qs = range(q.shape[0]) if queries is None else queries
    vm = valid_mask_dnf if disjunctive else valid_mask
    out_ids, out_d, nvalid = [], [], []
    for qi in qs:
        m = vm(dense, label_off, labels, pairs_of(con_off, con_attr, con_val, qi),
               n_dense, dense_vocab, label_vocab)
        ids = np.nonzero(m)[0]
        dd = dist64(x[ids], q[qi], metric)
        key = dd if metric == 0 else -dd
        order = np.lexsort((ids, key))[:k]
        r_ids = np.full(k, -1, dtype=np.int64)
        r_d = np.full(k, np.inf if metric == 0 else -np.inf)
        r_ids[:len(order)] = ids[order]
        r_d[:len(order)] = dd[order]
        out_ids.append(r_ids)
        out_d.append(r_d)
        nvalid.append(len(ids))
    return np.array(out_ids), np.array(out_d), np.array(nvalid)


def recall_at_k(found, truth, nvalid, k):
    """|found intersect truth| / min(k, |D_C|) per query (queries with an empty
    D_C count as 1 when nothing is returned)."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    r = np.zeros(found.shape[0])
    for i in range(found.shape[0]):
        denom = min(k, int(nvalid[i]))
        t = set(int(v) for v in truth[i, :k] if v >= 0)
        f = set(int(v) for v in found[i, :k] if v >= 0)
        r[i] = 1.0 if denom == 0 else len(t & f) / denom
    return r


def label_index(label_off, labels, n):
    """Inverted index of label sets: (starts, ids), the ids holding label l
    being ids[starts[l]:starts[l + 1]] in ascending order."""
    label_off = np.asarray(label_off, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    owner = np.repeat(np.arange(n, dtype=np.int64), np.diff(label_off))
    order = np.lexsort((owner, labels))
    vocab = int(labels.max()) + 1 if len(labels) else 0
    starts = np.zeros(vocab + 1, dtype=np.int64)
    np.add.at(starts, labels + 1, 1)
    return np.cumsum(starts), owner[order]


def topk64_labels(x, inv, metric, q, con_off, con_attr, con_val, k, label_attr, queries):
    """topk64 for label-only constraints through an inverted index: the valid
    set is the intersection of the constrained labels' id lists (Definition
    1); distances in FP64, ties to the smaller id.  Returns (ids, dists,
    |D_C|) for the given queries."""
    starts, ids_all = inv
    out_ids, out_d, nvalid = [], [], []
    n = x.shape[0]
    for qi in queries:
        pairs = pairs_of(con_off, con_attr, con_val, qi)
        valid = np.arange(n)
        for a, v in pairs:
            if a != label_attr or v < 0 or v + 1 >= len(starts):
                valid = np.zeros(0, dtype=np.int64)
                break
            valid = np.intersect1d(valid, ids_all[starts[v]:starts[v + 1]], assume_unique=True)
        dd = dist64(x[valid], q[qi], metric)
        key = dd if metric == 0 else -dd
        order = np.lexsort((valid, key))[:k]
        r_ids = np.full(k, -1, dtype=np.int64)
        r_d = np.full(k, np.inf if metric == 0 else -np.inf)
        r_ids[:len(order)] = valid[order]
        r_d[:len(order)] = dd[order]
        out_ids.append(r_ids)
        out_d.append(r_d)
        nvalid.append(len(valid))
    return np.array(out_ids), np.array(out_d), np.array(nvalid)
