"""Seeded synthetic workloads for CAPS filtered search.

This module only draws inputs: vectors, per-point attribute sets, query
vectors and query constraints.  It holds none of the method's arithmetic
(no partitioning, no distances, no ranking); both the CPU oracle and the
GPU library read what it produces.

Workload shapes follow the five configurations the build targets
(small Gaussian-mixture parity case; a SIFT1M-shaped integer corpus; an
angular corpus with label sets; the router's training set on the second
corpus; a 10M-point serving corpus).  The paper's own evaluation attaches
synthetic attributes to public corpora (Evaluation, "Datasets"); those
corpora are not available here and these generators stand in for them.

Random streams: numpy ``Generator(PCG64)`` seeded from
``SeedSequence(seed).spawn(4)`` -> (vectors, attributes, queries,
constraints).  Zipf(s) over a finite vocabulary V puts P(r) proportional
to (r+1)^-s for r = 0..V-1 (value 0 most frequent), sampled by inverse CDF.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BASE_SEED = 2308_15014


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray                      # (N, d) float32, row-major
    dense: Optional[np.ndarray]        # (N, L) uint32 or None
    dense_vocab: List[int]             # vocabulary size per dense attribute
    label_off: Optional[np.ndarray]    # (N+1,) int64 CSR offsets or None
    labels: Optional[np.ndarray]       # (nnz,) uint32 or None
    label_vocab: int                   # 0 when there are no labels
    q: np.ndarray                      # (Q, d) float32
    con_off: np.ndarray                # (Q+1,) int32 CSR over constraint pairs
    con_attr: np.ndarray               # (nc,) int32: dense attr index, or L for a label
    con_val: np.ndarray                # (nc,) int32
    metric: int                        # 0 squared L2, 1 inner product
    n_partitions: int                  # B
    aft_height: int                    # h
    kmeans_iters: int
    k: int
    nprobe: int
    seed: int
    selectivity: Optional[np.ndarray] = None   # |D_C|/N per query when known

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_q(self) -> int:
        return int(self.q.shape[0])

    @property
    def n_dense(self) -> int:
        return 0 if self.dense is None else int(self.dense.shape[1])


def zipf_cdf(vocab: int, s: float) -> np.ndarray:
    w = (np.arange(1, vocab + 1, dtype=np.float64)) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_draw(rng: np.random.Generator, cdf: np.ndarray, size) -> np.ndarray:
    u = rng.random(size)
    v = np.searchsorted(cdf, u, side="right")
    return np.minimum(v, len(cdf) - 1).astype(np.uint32)


def draw_dense(rng, n, vocabs, s):
    cols = [zipf_draw(rng, zipf_cdf(v, s), n) for v in vocabs]
    return np.stack(cols, axis=1).astype(np.uint32)


def draw_label_sets(rng, n, vocab, s, max_size=8):
    """Per point: size ~ U{1..max_size}; labels Zipf(s) without replacement
    (a duplicate draw is drawn again)."""
    cdf = zipf_cdf(vocab, s)
    size = rng.integers(1, max_size + 1, size=n)
    lab = zipf_draw(rng, cdf, (n, max_size)).astype(np.int64)
    for c in range(1, max_size):
        active = size > c
        while True:
            dup = np.zeros(n, dtype=bool)
            for e in range(c):
                dup |= lab[:, c] == lab[:, e]
            dup &= active
            cnt = int(dup.sum())
            if cnt == 0:
                break
            lab[dup, c] = zipf_draw(rng, cdf, cnt)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(size)
    mask = np.arange(max_size)[None, :] < size[:, None]
    labels = lab[mask].astype(np.uint32)
    return off, labels


class _DenseCounter:
    """|{i : a_i[attr]=val for every constrained attr}| from a joint count
    table (used only to keep queries inside a selectivity band)."""

    def __init__(self, dense, vocabs):
        self.vocabs = list(vocabs)
        flat = np.zeros(dense.shape[0], dtype=np.int64)
        for i, v in enumerate(vocabs):
            flat = flat * v + dense[:, i].astype(np.int64)
        total = int(np.prod(vocabs))
        self.table = np.bincount(flat, minlength=total).reshape(vocabs)

    def count(self, pairs):
        idx = [slice(None)] * len(self.vocabs)
        for a, v in pairs:
            if idx[a] != slice(None) and idx[a] != v:
                return 0
            idx[a] = v
        return int(self.table[tuple(idx)].sum())


class _LabelCounter:
    """Counts points holding every label of a set, from posting lists."""

    def __init__(self, off, labels, n):
        self.n = n
        owner = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
        order = np.argsort(labels, kind="stable")
        self.own_sorted = owner[order]
        # label l's owners are own_sorted[start[l]:start[l + 1]]
        counts = np.bincount(labels, minlength=int(labels.max()) + 1 if len(labels) else 1)
        self.start = np.concatenate([[0], np.cumsum(counts)])

    def posting(self, lab):
        if lab < 0 or lab + 1 >= len(self.start):
            return self.own_sorted[:0]
        return self.own_sorted[self.start[lab]:self.start[lab + 1]]

    def ids(self, labs):
        if not labs:
            return None
        lists = sorted((self.posting(l) for l in labs), key=len)
        cur = lists[0]
        for p in lists[1:]:
            if cur.size == 0:
                break
            cur = np.intersect1d(cur, p, assume_unique=True)
        return cur


class _BitCounter:
    """|{i : every pair (attr, val) holds}| for dense values and labels from
    packed bitsets: one per dense value and per label with a long posting
    list; a pair set with a short posting list is counted by testing those
    ids against the other pairs' bitsets.  (Used only to keep queries inside
    a selectivity band; the counts equal a direct evaluation.)"""

    def __init__(self, dense, vocabs, off, labels, n, long_posting=20_000):
        self.n, self.nd = n, len(vocabs)
        self.words = (n + 63) // 64
        self.dense_bits = {}
        for a, v in enumerate(vocabs):
            col = dense[:, a]
            for val in range(v):
                self.dense_bits[(a, val)] = self._pack(np.flatnonzero(col == val))
        self.lab = _LabelCounter(off, labels, n)
        counts = np.bincount(labels, minlength=int(labels.max()) + 1 if len(labels) else 1)
        self.label_bits = {int(l): self._pack(self.lab.posting(l)) for l in np.flatnonzero(counts >= long_posting)}

    def _pack(self, ids):
        bits = np.zeros(self.words * 64, dtype=bool)
        bits[ids] = True
        return np.packbits(bits, bitorder="little").view(np.uint64)

    def _bits(self, a, v):
        return self.dense_bits[(a, v)] if a < self.nd else self.label_bits.get(v)

    def count(self, pairs):
        pairs = list(dict.fromkeys(pairs))
        dense_vals = {}
        for a, v in pairs:
            if a < self.nd:
                if dense_vals.setdefault(a, v) != v:
                    return 0
        short = [v for a, v in pairs if a >= self.nd and v not in self.label_bits]
        if short:
            ids = self.lab.ids(short)
            if ids.size == 0:
                return 0
            keep = np.ones(ids.size, dtype=bool)
            for a, v in pairs:
                if a >= self.nd and v in short:
                    continue
                b = self._bits(a, v)
                keep &= ((b[ids >> 6] >> (ids & 63).astype(np.uint64)) & np.uint64(1)).astype(bool)
            return int(keep.sum())
        acc = None
        for a, v in pairs:
            b = self._bits(a, v)
            acc = b.copy() if acc is None else acc & b
        return self.n if acc is None else int(np.bitwise_count(acc).sum())


def draw_constraints(rng, n_q, n, dense, label_off, labels, cmin, cmax,
                     band=None, counter=None):
    """Each query copies c ~ U{cmin..cmax} attributes (dense values and/or
    labels) of a uniformly drawn database point, chosen without replacement.
    When ``band`` = (lo, hi) is given, a draw whose |D_C|/N falls outside the
    band is discarded and drawn again."""
    n_dense = 0 if dense is None else dense.shape[1]
    off = [0]
    attrs: List[int] = []
    vals: List[int] = []
    sel = np.zeros(n_q, dtype=np.float64)
    for qi in range(n_q):
        for _attempt in range(100000):
            pt = int(rng.integers(n))
            pool = [(a, int(dense[pt, a])) for a in range(n_dense)]
            if labels is not None:
                pool += [(n_dense, int(l)) for l in labels[label_off[pt]:label_off[pt + 1]]]
            c = int(rng.integers(cmin, cmax + 1))
            c = min(c, len(pool))
            pick = rng.choice(len(pool), size=c, replace=False)
            pairs = [pool[j] for j in sorted(pick)]
            if counter is None:
                break
            cnt = counter(pairs)
            frac = cnt / n
            sel[qi] = frac
            if band is None or (band[0] <= frac <= band[1]):
                break
        else:
            raise RuntimeError("selectivity band unreachable")
        for a, v in pairs:
            attrs.append(a)
            vals.append(v)
        off.append(len(attrs))
    return (np.asarray(off, dtype=np.int32), np.asarray(attrs, dtype=np.int32),
            np.asarray(vals, dtype=np.int32), sel)


OR_ATTR = -1   # constraint attribute that separates the AND-terms of a disjunctive query


def draw_disjunctions(rng, n_q, n, dense, label_off, labels, tmin, tmax, cmin, cmax):
    """Disjunctive queries: t ~ U{tmin..tmax} AND-terms, each drawn as by
    draw_constraints (pairs copied from its own random database point), joined
    by (OR_ATTR, 0) separators."""
    off = [0]
    attrs: List[int] = []
    vals: List[int] = []
    for _ in range(n_q):
        t = int(rng.integers(tmin, tmax + 1))
        co, ca, cv, _sel = draw_constraints(rng, t, n, dense, label_off, labels, cmin, cmax)
        for j in range(t):
            if j:
                attrs.append(OR_ATTR)
                vals.append(0)
            attrs.extend(ca[co[j]:co[j + 1]].tolist())
            vals.extend(cv[co[j]:co[j + 1]].tolist())
        off.append(len(attrs))
    return (np.asarray(off, dtype=np.int32), np.asarray(attrs, dtype=np.int32),
            np.asarray(vals, dtype=np.int32))


def _streams(seed):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]


def make_c1(n=10_000, n_q=100, seed=None) -> Workload:
    """Gaussian mixture: 16 means ~ N(0, 4I), points = mean + N(0, I), d=32.
    Three dense attributes (10/10/20) Zipf(1.0).  Queries are database points
    plus N(0, 0.1 I); each carries 1-2 constraints copied from an independently
    drawn database point.  B=32, h=2, 10 Lloyd iterations, k=10, nprobe=4, L2."""
    seed = BASE_SEED + 1 if seed is None else seed
    rv, ra, rq, rc = _streams(seed)
    d = 32
    means = rv.normal(0.0, 2.0, size=(16, d))
    comp = rv.integers(16, size=n)
    x = (means[comp] + rv.normal(0.0, 1.0, size=(n, d))).astype(np.float32)
    vocab = [10, 10, 20]
    dense = draw_dense(ra, n, vocab, 1.0)
    src = rq.integers(n, size=n_q)
    q = (x[src].astype(np.float64) + rq.normal(0.0, np.sqrt(0.1), size=(n_q, d))).astype(np.float32)
    cnt = _DenseCounter(dense, vocab)
    co, ca, cv, sel = draw_constraints(rc, n_q, n, dense, None, None, 1, 2, None, cnt.count)
    return Workload("c1", x, dense, vocab, None, None, 0, q, co, ca, cv, 0,
                    32, 2, 10, 10, 4, seed, sel)


def make_c2(n=1_000_000, n_q=10_000, seed=None, band=(0.001, 0.30), n_partitions=1024) -> Workload:
    """SIFT1M-shaped: uniform integers 0..255 stored as float32, d=128.
    Three dense attributes (10/50/200) Zipf(1.0).  Queries: uniform integers,
    1-3 constraints, selectivity |D_C|/N within ``band``.  B=1024, h=2."""
    seed = BASE_SEED + 2 if seed is None else seed
    rv, ra, rq, rc = _streams(seed)
    d = 128
    x = rv.integers(0, 256, size=(n, d), dtype=np.int32).astype(np.float32)
    vocab = [10, 50, 200]
    dense = draw_dense(ra, n, vocab, 1.0)
    q = rq.integers(0, 256, size=(n_q, d), dtype=np.int32).astype(np.float32)
    cnt = _DenseCounter(dense, vocab)
    co, ca, cv, sel = draw_constraints(rc, n_q, n, dense, None, None, 1, 3, band, cnt.count)
    return Workload("c2", x, dense, vocab, None, None, 0, q, co, ca, cv, 0,
                    n_partitions, 2, 10, 10, 32, seed, sel)


def make_c2_queries(n_q, seed, n=1_000_000, band=(0.001, 0.30)):
    """Extra query sets drawn from the c2 query generator with another seed
    (router training and held-out sets).  The corpus itself is unchanged."""
    base = make_c2(n=n, n_q=1, band=band)
    _rv, _ra, rq, rc = _streams(seed)
    q = rq.integers(0, 256, size=(n_q, base.d), dtype=np.int32).astype(np.float32)
    cnt = _DenseCounter(base.dense, base.dense_vocab)
    co, ca, cv, sel = draw_constraints(rc, n_q, base.n, base.dense, None, None, 1, 3, band, cnt.count)
    return q, co, ca, cv, sel


def make_c2_train_queries(n_q, seed, base: Workload, band=(0.001, 0.30)):
    """Large query sets in the shape of c2's (uniform integer vectors, 1-3
    constraints copied from a random point's dense attributes, |D_C|/N in
    ``band``), drawn in vectorised rounds: every round draws a candidate for
    each missing query and keeps those inside the band.  For router training
    sets of millions of queries; the per-query generator above is the
    reference for the benchmark's own query set."""
    _rv, _ra, rq, rc = _streams(seed)
    n, nd = base.n, base.dense.shape[1]
    q = rq.integers(0, 256, size=(n_q, base.d), dtype=np.int32).astype(np.float32)
    vocabs = list(base.dense_vocab)
    cnt = _DenseCounter(base.dense, vocabs)
    # count tables of every attribute subset (bit a set: attribute a constrained)
    marg = {}
    for sub in range(1 << nd):
        keep = tuple(a for a in range(nd) if not (sub >> a) & 1)
        marg[sub] = cnt.table.sum(axis=keep) if keep else cnt.table
    nc = np.zeros(n_q, dtype=np.int64)
    attr = np.zeros((n_q, nd), dtype=bool)
    val = np.zeros((n_q, nd), dtype=np.int64)
    todo = np.arange(n_q)
    while len(todo):
        k = len(todo)
        pt = rc.integers(n, size=k)
        c = np.minimum(rc.integers(1, 4, size=k), nd)
        order = np.argsort(rc.random((k, nd)), axis=1)
        chosen = np.zeros((k, nd), dtype=bool)
        np.put_along_axis(chosen, order, np.arange(nd)[None, :] < c[:, None], axis=1)
        v = base.dense[pt].astype(np.int64)
        sub = (chosen * (1 << np.arange(nd))[None, :]).sum(axis=1)
        counts = np.zeros(k, dtype=np.int64)
        for sv in np.unique(sub):
            rows = np.nonzero(sub == sv)[0]
            sel_attrs = [a for a in range(nd) if (sv >> a) & 1]
            counts[rows] = marg[int(sv)][tuple(v[rows, a] for a in sel_attrs)]
        frac = counts / n
        ok = (frac >= band[0]) & (frac <= band[1])
        acc = todo[ok]
        attr[acc] = chosen[ok]
        val[acc] = v[ok]
        nc[acc] = c[ok]
        todo = todo[~ok]
    co = np.concatenate([[0], np.cumsum(nc)]).astype(np.int32)
    rows, cols = np.nonzero(attr)            # row-major: attributes ascending per query
    ca = cols.astype(np.int32)
    cv = val[rows, cols].astype(np.int32)
    return q, co, ca, cv


def make_absence_queries(n_q, seed, base: Workload, absence: float):
    """Queries in the shape of the paper's absence-fraction ablation (Section
    6 "Varying number of attributes"): uniform integer vectors as the base
    corpus's; each query copies the attribute values of a random database
    point and drops each attribute independently with probability
    `absence` (0: every attribute constrained; 1: no constraint)."""
    _rv, _ra, rq, rc = _streams(seed)
    n, nd = base.n, base.dense.shape[1]
    q = rq.integers(0, 256, size=(n_q, base.d), dtype=np.int32).astype(np.float32)
    pt = rc.integers(n, size=n_q)
    keep = rc.random((n_q, nd)) >= absence
    rows, cols = np.nonzero(keep)
    co = np.concatenate([[0], np.cumsum(keep.sum(axis=1))]).astype(np.int32)
    return q, co, cols.astype(np.int32), base.dense[pt[rows], cols].astype(np.int32)


def make_c3(n=5_000_000, n_q=10_000, seed=None, n_partitions=4096) -> Workload:
    """Angular corpus: g/|g| with g ~ N(0, I), d=96, inner product.  Each
    point holds 1-8 labels from a vocabulary of 1000, Zipf(1.1).  Queries:
    fresh unit Gaussians with 1-4 label constraints.  B=4096, h=4."""
    seed = BASE_SEED + 3 if seed is None else seed
    rv, ra, rq, rc = _streams(seed)
    d = 96
    g = rv.standard_normal(size=(n, d))
    x = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    del g
    off, labels = draw_label_sets(ra, n, 1000, 1.1)
    gq = rq.standard_normal(size=(n_q, d))
    q = (gq / np.linalg.norm(gq, axis=1, keepdims=True)).astype(np.float32)
    co, ca, cv, sel = draw_constraints(rc, n_q, n, None, off, labels, 1, 4, None, None)
    return Workload("c3", x, None, [], off, labels, 1000, q, co, ca, cv, 1,
                    n_partitions, 4, 10, 10, 64, seed, None)


def make_c5(n=10_000_000, n_q=10_000, seed=None, n_partitions=8192,
            band=(0.0001, 0.50)) -> Workload:
    """Serving corpus: c2-style integer vectors (exact in FP16), d=128, three
    dense attributes (10/50/200, Zipf 1.0) plus label sets of 1-8 labels from
    5000, Zipf(1.1).  Queries: 1-4 constraints mixing both kinds, selectivity
    within ``band``.  B=8192, h=4."""
    seed = BASE_SEED + 5 if seed is None else seed
    rv, ra, rq, rc = _streams(seed)
    d = 128
    x = rv.integers(0, 256, size=(n, d), dtype=np.int32).astype(np.float32)
    vocab = [10, 50, 200]
    dense = draw_dense(ra, n, vocab, 1.0)
    off, labels = draw_label_sets(ra, n, 5000, 1.1)
    q = rq.integers(0, 256, size=(n_q, d), dtype=np.int32).astype(np.float32)
    cnt = _BitCounter(dense, vocab, off, labels, n)
    co, ca, cv, sel = draw_constraints(rc, n_q, n, dense, off, labels, 1, 4, band, cnt.count)
    return Workload("c5", x, dense, vocab, off, labels, 5000, q, co, ca, cv, 0,
                    n_partitions, 4, 10, 10, 64, seed, sel)


def make_wide(n_attrs, p_select, n=1_000_000, n_q=10_000, seed=None, vocab=10, n_partitions=1024,
              max_constraints=8) -> Workload:
    """Larger attribute lengths (the paper's appendix, L = 3 / 10 / 100 with
    per-query selection probability 1 / 0.3 / 0.03) as a label-style
    workload at the 1M-point scale: c2's integer vectors; every point holds
    L attributes, attribute a with a value v ~ Zipf(1.0) over `vocab`,
    stored as label a * vocab + v (so each point has exactly L labels).  A
    query copies the attributes of a random database point and keeps each
    with probability `p_select` (drawn again when more than
    `max_constraints` are kept).  B=1024, h=2."""
    seed = BASE_SEED + 7 + n_attrs if seed is None else seed
    base = make_c2(n=n, n_q=1)
    _rv, ra, rq, rc = _streams(seed)
    vals = draw_dense(ra, n, [vocab] * n_attrs, 1.0).astype(np.int64)
    labels = (vals + vocab * np.arange(n_attrs)[None, :]).astype(np.uint32).reshape(-1)
    off = (np.arange(n + 1, dtype=np.int64) * n_attrs)
    q = rq.integers(0, 256, size=(n_q, base.d), dtype=np.int32).astype(np.float32)
    co, ca, cv = [0], [], []
    for _ in range(n_q):
        pt = int(rc.integers(n))
        while True:
            keep = np.flatnonzero(rc.random(n_attrs) < p_select)
            if len(keep) <= max_constraints:
                break
        ca.extend([0] * len(keep))
        cv.extend(labels[pt * n_attrs + keep].tolist())
        co.append(len(ca))
    return Workload(f"wide{n_attrs}", base.x, None, [], off, labels, vocab * n_attrs, q,
                    np.asarray(co, np.int32), np.asarray(ca, np.int32), np.asarray(cv, np.int32), 0,
                    n_partitions, 2, 10, 10, 32, seed, None)


def make_c5_queries(n_q, seed, base: Workload):
    """Query sets in the shape of c5's (uniform integer vectors, 1-4
    constraints copied from a random point's dense attributes and labels)
    without the selectivity redraw, for router training sets."""
    _rv, _ra, rq, rc = _streams(seed)
    q = rq.integers(0, 256, size=(n_q, base.d), dtype=np.int32).astype(np.float32)
    co, ca, cv, _sel = draw_constraints(rc, n_q, base.n, base.dense, base.label_off, base.labels, 1, 4)
    return q, co, ca, cv


def make_tiny(rng_seed, n, d, n_q, vocabs=(3, 4), label_vocab=0, metric=0,
              b=4, h=2, cmin=0, cmax=2, integer=False, max_labels=4):
    """Small random workloads for exhaustive and property tests."""
    rv, ra, rq, rc = _streams(rng_seed)
    if integer:
        x = rv.integers(0, 8, size=(n, d)).astype(np.float32)
        q = rq.integers(0, 8, size=(n_q, d)).astype(np.float32)
    else:
        x = rv.normal(size=(n, d)).astype(np.float32)
        q = rq.normal(size=(n_q, d)).astype(np.float32)
    dense = draw_dense(ra, n, list(vocabs), 1.0) if vocabs else None
    if label_vocab:
        off, labels = draw_label_sets(ra, n, label_vocab, 1.1, max_size=max_labels)
    else:
        off, labels = None, None
    co, ca, cv, sel = draw_constraints(rc, n_q, n, dense, off, labels, cmin, cmax, None, None)
    return Workload("tiny", x, dense, list(vocabs) if vocabs else [], off, labels,
                    label_vocab, q, co, ca, cv, metric, b, h, 5, 5, 2, rng_seed, None)


def make_routed(n=40_000, n_q=4000, seed=None, n_clusters=64, d=32, n_vals=8, purity=0.9):
    """A workload where the filter, not the query vector alone, decides which
    partitions hold the answers: a Gaussian mixture (means ~ N(0, 9I), unit
    noise) whose single dense attribute equals cluster % n_vals with
    probability `purity` (uniform otherwise).  Each query is a point near a
    random cluster mean with one constraint whose value is drawn
    independently of that cluster, so its filtered neighbours sit mostly in
    other clusters.  B = n_clusters, h = 1."""
    seed = BASE_SEED + 6 if seed is None else seed
    rv, ra, rq, rc = _streams(seed)
    means = rv.normal(0.0, 3.0, size=(n_clusters, d))
    comp = rv.integers(n_clusters, size=n)
    x = (means[comp] + rv.normal(0.0, 1.0, size=(n, d))).astype(np.float32)
    keep = ra.random(n) < purity
    attr = np.where(keep, comp % n_vals, ra.integers(n_vals, size=n)).astype(np.uint32)
    qc = rq.integers(n_clusters, size=n_q)
    q = (means[qc] + rq.normal(0.0, 1.0, size=(n_q, d))).astype(np.float32)
    co = np.arange(n_q + 1, dtype=np.int32)
    ca = np.zeros(n_q, dtype=np.int32)
    cv = rc.integers(n_vals, size=n_q).astype(np.int32)
    return Workload("routed", x, attr[:, None], [n_vals], None, None, 0, q, co, ca, cv, 0,
                    n_clusters, 1, 10, 10, 4, seed, None)


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c5": make_c5, "routed": make_routed}
