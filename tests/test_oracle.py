"""Pins for the CPU oracle against what the paper and mathematics fix.

Every check here compares the oracle with something other than itself:
published generator outputs, a hand-worked example of Algorithm 1, closed
forms (B = 1 k-means is the mean), textbook invariants (Lloyd's objective
does not increase; the AFT sub-partitions are a disjoint cover), exhaustive
FP64 brute force on small inputs, and special cases that reduce to library
routines (unconstrained search with every partition probed is exact kNN).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ref64

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed, **kw):
    return synth.make_tiny(seed, **kw)


# ------------------------------------------------------------- sampler
def test_splitmix64_published_vectors(orc):
    for line in open(os.path.join(GOLD, "splitmix64_vectors.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        seed, vals = line.split(":")
        want = [int(v) for v in vals.split()]
        got = [int(v) for v in orc.splitmix64(int(seed), len(want))]
        assert got == want


def test_init_ids_hand_worked(orc):
    # partial Fisher-Yates on the published generator outputs, worked by hand
    for line in open(os.path.join(GOLD, "init_ids_worked.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, vals = line.split(":")
        seed, n, b = (int(v) for v in head.split())
        assert orc.init_ids(seed, n, b).tolist() == [int(v) for v in vals.split()], head


def test_init_ids_distinct_in_range(orc):
    for seed in range(20):
        ids = orc.init_ids(seed, 1000, 64)
        assert len(set(ids.tolist())) == 64
        assert ids.min() >= 0 and ids.max() < 1000
    full = orc.init_ids(7, 50, 50)
    assert sorted(full.tolist()) == list(range(50))


def test_init_ids_roughly_uniform(orc):
    hits = np.zeros(20)
    for seed in range(2000):
        hits[orc.init_ids(seed, 20, 3)] += 1
    # each id is picked with probability 3/20 per draw: 300 expected
    assert np.all(np.abs(hits - 300) < 80)


# ------------------------------------------------------------- k-means
def test_kmeans_b1_is_fp64_mean_rounded(orc):
    rng = np.random.default_rng(0)
    x = rng.integers(-50, 50, size=(301, 7)).astype(np.float32)
    cent, a = orc.kmeans(x, 1, 3, init=np.array([5], dtype=np.int32))
    # integer data: the FP64 sum is exact in any order
    want = (x.astype(np.float64).sum(0) / x.shape[0]).astype(np.float32)
    assert np.array_equal(cent[0], want)
    assert np.all(a == 0)


def test_objective_hand_value(orc):
    # three points, one centroid at the origin: 0 + 2^2 + 4^2
    x = np.array([[0, 0], [2, 0], [0, 4]], np.float32)
    assert orc.objective(x, np.zeros((1, 2), np.float32), np.zeros(3, np.int32)) == 20.0
    # two clusters: distances 1 and 1 to c0, 9 to c1
    x = np.array([[1, 0], [-1, 0], [5, 3]], np.float32)
    c = np.array([[0, 0], [5, 0]], np.float32)
    assert orc.objective(x, c, np.array([0, 0, 1], np.int32)) == 11.0


def test_objective_koenig_huygens(orc):
    # for one cluster, sum |x - c|^2 = sum |x - mean|^2 + n |c - mean|^2 and
    # sum |x - mean|^2 = sum |x|^2 - n |mean|^2 (integer data with an
    # integer mean: every quantity is exact in FP64)
    rng = np.random.default_rng(11)
    x = rng.integers(-30, 30, size=(40, 5)).astype(np.int64)
    x[-1] -= x.sum(0) - 40 * rng.integers(-3, 3, size=5)   # force an integer mean
    mean = x.sum(0) // 40
    assert np.array_equal(mean * 40, x.sum(0))
    a = np.zeros(40, np.int32)
    within = orc.objective(x.astype(np.float32), mean[None].astype(np.float32), a)
    assert within == float((x * x).sum() - 40 * (mean * mean).sum())
    for c in (mean + np.array([1, 0, -2, 3, 0]), mean - 7):
        got = orc.objective(x.astype(np.float32), c[None].astype(np.float32), a)
        assert got == within + 40 * float(((c - mean) ** 2).sum())


def test_kmeans_objective_nonincreasing(orc):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2000, 8)).astype(np.float32)
    init = orc.init_ids(3, 2000, 12)
    prev = None
    for it in range(0, 8):
        cent, a = orc.kmeans(x, 12, it, init=init)
        obj = orc.objective(x, cent, a)
        if prev is not None:
            assert obj <= prev * (1 + 1e-9)
        prev = obj


def test_kmeans_separated_mixture_recovered(orc):
    rng = np.random.default_rng(2)
    means = np.array([[100, 0], [0, 100], [-100, 0], [0, -100]], dtype=np.float64)
    comp = rng.integers(4, size=400)
    x = (means[comp] + rng.normal(size=(400, 2))).astype(np.float32)
    # one init point from each component
    init = np.array([np.nonzero(comp == c)[0][0] for c in range(4)], dtype=np.int32)
    cent, a = orc.kmeans(x, 4, 5, init=init)
    assert np.array_equal(a, comp)
    for c in range(4):
        want = (x[comp == c].astype(np.float64).sum(0) / (comp == c).sum()).astype(np.float32)
        # sums of non-integer data: FP64 ascending-order sum vs numpy pairwise
        # sum agree to far below FP32 resolution
        assert np.allclose(cent[c], want, rtol=0, atol=1e-5)


def test_kmeans_assignment_is_argmin(orc):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3000, 16)).astype(np.float32)
    c = rng.normal(size=(40, 16)).astype(np.float32)
    a = orc.assign(x, c, 0)
    d64 = ((x.astype(np.float64)[:, None, :] - c.astype(np.float64)[None]) ** 2).sum(-1)
    best = d64.min(1)
    chosen = d64[np.arange(len(x)), a]
    # the FP32 expansion |c|^2 - 2x.c can only swap near-ties
    assert np.all(chosen <= best + 1e-3 * (1 + best))
    assert np.mean(a == d64.argmin(1)) > 0.995
    # inner product: argmax of the dot product
    a_ip = orc.assign(x, c, 1)
    ip = x.astype(np.float64) @ c.astype(np.float64).T
    assert np.mean(a_ip == ip.argmax(1)) > 0.995


def test_kmeans_empty_cluster_keeps_centroid(orc):
    rng = np.random.default_rng(4)
    x = rng.normal(size=(100, 3)).astype(np.float32)
    c0 = x[[0, 0, 5]].copy()                     # centroid 1 duplicates 0
    a = orc.assign(x, c0, 0)
    assert not np.any(a == 1)                      # ties go to the smaller id
    c1 = orc.update(x, a, c0, 0)
    assert np.array_equal(c1[1], x[0])             # empty cluster keeps its centroid
    assert not np.array_equal(c1[0], x[0])


def test_kmeans_spherical_unit_norm(orc):
    rng = np.random.default_rng(5)
    g = rng.normal(size=(500, 6))
    x = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    cent, a = orc.kmeans(x, 5, 4, metric=1, init=np.arange(5, dtype=np.int32))
    nrm = np.linalg.norm(cent.astype(np.float64), axis=1)
    assert np.all(np.abs(nrm - 1) < 1e-6)


# ------------------------------------------------------------- AFT / CSR
def _worked():
    g = json.load(open(os.path.join(GOLD, "aft_worked_example.json")))
    dense = np.array(g["dense"], dtype=np.uint32)
    return g, dense


def test_aft_hand_worked_example(orc):
    g, dense = _worked()
    tk = orc.tokens_of(dense, g["dense_vocab"], None, None, 0)
    a = np.zeros(len(dense), dtype=np.int32)
    tags, level = orc.aft(a, 1, g["h"], tk)
    assert tags.ravel().tolist() == g["tags"]
    assert level.tolist() == g["level"]
    perm, offs = orc.csr(a, level, 1, g["h"], np.asarray(dense))
    assert perm.tolist() == g["perm"]
    assert offs.tolist() == g["offs"]


@pytest.mark.parametrize("rule", [0, 1])
def test_subpartition_choice_hand_worked(orc, rule):
    g, dense = _worked()
    n = len(dense)
    x = np.arange(n * 2, dtype=np.float32).reshape(n, 2)
    idx = orc.build_index(x, dense, g["dense_vocab"], None, None, 0, metric=0, b=1,
                          h=g["h"], iters=0, seed=0, init=np.array([0], dtype=np.int32))
    qs = g["queries"]
    con_off = np.cumsum([0] + [len(qq["pairs"]) for qq in qs]).astype(np.int32)
    ca = np.array([p[0] for qq in qs for p in qq["pairs"]], dtype=np.int32)
    cv = np.array([p[1] for qq in qs for p in qq["pairs"]], dtype=np.int32)
    q = np.zeros((len(qs), 2), dtype=np.float32)
    r = orc.search(idx, q, con_off, ca, cv, k=8, m=1, rule=rule)
    for i, qq in enumerate(qs):
        if rule == 0:
            assert int(r.masks[i, 0]) == qq["mask"]
            assert int(r.n_cand[i]) == qq["n_cand"]
            assert sorted(v for v in r.ids[i].tolist() if v >= 0) == qq["valid"]
        else:
            assert int(r.masks[i, 0]) == qq["literal_mask"]
    if rule == 1:
        # the literal rule misses point 3 for {A0=c}: it is the reason for
        # the exact rule
        assert 3 not in r.ids[1].tolist()


@pytest.mark.parametrize("rule", [0, 1])
def test_disjunctive_choice_hand_worked(orc, rule):
    g, dense = _worked()
    n = len(dense)
    x = np.arange(n * 2, dtype=np.float32).reshape(n, 2)
    idx = orc.build_index(x, dense, g["dense_vocab"], None, None, 0, metric=0, b=1,
                          h=g["h"], iters=0, seed=0, init=np.array([0], dtype=np.int32))
    qs = g["or_queries"]
    con_off = np.cumsum([0] + [len(qq["pairs"]) for qq in qs]).astype(np.int32)
    ca = np.array([p[0] for qq in qs for p in qq["pairs"]], dtype=np.int32)
    cv = np.array([p[1] for qq in qs for p in qq["pairs"]], dtype=np.int32)
    q = np.zeros((len(qs), 2), dtype=np.float32)
    r = orc.search(idx, q, con_off, ca, cv, k=8, m=1, rule=rule, disjunctive=True)
    for i, qq in enumerate(qs):
        if rule == 0:
            assert int(r.masks[i, 0]) == qq["mask"], i
            assert int(r.n_cand[i]) == qq["n_cand"], i
            assert sorted(v for v in r.ids[i].tolist() if v >= 0) == qq["valid"], i
        else:
            assert int(r.masks[i, 0]) == qq["literal_mask"], i
    # without the disjunctive reading the separator is an invalid pair
    r = orc.search(idx, q, con_off, ca, cv, k=8, m=1)
    assert (r.ids == -1).all() and (r.masks == 0).all()


def _or_workload(seed, **kw):
    w = _tiny(seed, **kw)
    rng = np.random.default_rng(seed + 1)
    co, ca, cv = synth.draw_disjunctions(rng, w.n_q, w.n, w.dense, w.label_off, w.labels, 1, 3, 0, 2)
    w.con_off, w.con_attr, w.con_val = co, ca, cv
    return w


OR_CASES = [
    dict(n=700, d=6, n_q=60, vocabs=(3, 5), label_vocab=0, b=6, h=2),
    dict(n=900, d=9, n_q=60, vocabs=(4,), label_vocab=12, b=5, h=3, integer=True),
    dict(n=800, d=5, n_q=60, vocabs=(), label_vocab=9, b=4, h=1, metric=1),
]


@pytest.mark.parametrize("case", OR_CASES)
def test_disjunctive_all_partitions_equals_bruteforce(orc, case):
    w = _or_workload(61, **case)
    idx = orc.build_from_workload(w, iters=2)
    r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, 7, w.n_partitions, disjunctive=True)
    bf = orc.bruteforce(w.x, idx.tk, w.metric, w.q, w.con_off, w.con_attr, w.con_val, 7, disjunctive=True)
    assert np.array_equal(r.ids, bf.ids)
    assert np.array_equal(r.dist.view(np.uint32), bf.dist.view(np.uint32))
    assert np.array_equal(r.n_surv, bf.n_surv)


@pytest.mark.parametrize("case", OR_CASES)
def test_disjunction_is_union_of_its_terms(orc, case):
    """The top k of T1 or T2 is the top k of the two terms' own top-k lists
    merged: checked against AND-only searches of each term."""
    w = _or_workload(62, **case)
    tk = orc.tokens_of(w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab)
    k = 6
    bf = orc.bruteforce(w.x, tk, w.metric, w.q, w.con_off, w.con_attr, w.con_val, k, disjunctive=True)
    for i in range(w.n_q):
        pairs = ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i)
        terms, cur = [], []
        for a, v in pairs:
            if a == -1:
                terms.append(cur)
                cur = []
            else:
                cur.append((a, v))
        terms.append(cur)
        hits = {}
        for t in terms:
            co = np.array([0, len(t)], np.int32)
            ca = np.array([a for a, _ in t], np.int32)
            cv = np.array([v for _, v in t], np.int32)
            r = orc.bruteforce(w.x, tk, w.metric, w.q[i:i + 1], co, ca, cv, k)
            for a, dd in zip(r.ids[0], r.dist[0]):
                if a >= 0:
                    hits[int(a)] = float(dd)
        key = (lambda kv: (kv[1], kv[0])) if w.metric == 0 else (lambda kv: (-kv[1], kv[0]))
        want = [a for a, _ in sorted(hits.items(), key=key)][:k]
        assert [int(a) for a in bf.ids[i] if a >= 0] == want, i


def test_disjunctive_bruteforce_matches_fp64(orc):
    w = _or_workload(63, n=1500, d=12, n_q=50, vocabs=(3, 4), label_vocab=10, b=4, h=2, integer=True)
    tk = orc.tokens_of(w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab)
    bf = orc.bruteforce(w.x, tk, 0, w.q, w.con_off, w.con_attr, w.con_val, 10, disjunctive=True)
    ids64, _, nv = ref64.topk64(w.x, w.dense, w.label_off, w.labels, w.dense_vocab, w.label_vocab, 0, w.q,
                                w.con_off, w.con_attr, w.con_val, 10, disjunctive=True)
    assert np.array_equal(bf.ids, ids64)        # integer data: FP32 distances are exact
    assert np.array_equal(bf.n_surv, nv)


def test_single_term_disjunction_is_the_conjunction(orc):
    w = _tiny(64, n=800, d=7, n_q=40, vocabs=(3, 4), label_vocab=8, b=5, h=2, cmin=0, cmax=3)
    idx = orc.build_from_workload(w, iters=2)
    a = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, 5, 3)
    b = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, 5, 3, disjunctive=True)
    for u, v in ((a.ids, b.ids), (a.masks, b.masks), (a.n_cand, b.n_cand), (a.n_surv, b.n_surv)):
        assert np.array_equal(u, v)


def test_insert_hand_worked(orc):
    g, dense = _worked()
    n = len(dense)
    x = np.arange(n * 2, dtype=np.float32).reshape(n, 2)
    idx = orc.build_index(x, dense, g["dense_vocab"], None, None, 0, metric=0, b=1,
                          h=g["h"], iters=0, seed=0, init=np.array([0], dtype=np.int32))
    new = np.array(g["inserts"], dtype=np.uint32)
    iy = orc.insert(idx, np.zeros((len(new), 2), np.float32), new, None, None)
    assert iy.level[n:].tolist() == g["insert_level"]
    assert iy.perm.tolist() == g["insert_perm"]
    assert iy.offs.tolist() == g["insert_offs"]
    assert np.array_equal(iy.tags, idx.tags) and np.array_equal(iy.centroids, idx.centroids)


@pytest.mark.parametrize("case", [
    dict(n=1200, d=8, n_q=40, vocabs=(3, 5), label_vocab=0, b=7, h=2),
    dict(n=1500, d=6, n_q=40, vocabs=(4,), label_vocab=12, b=6, h=3, integer=True),
    dict(n=1000, d=5, n_q=40, vocabs=(), label_vocab=9, b=5, h=4, metric=1),
])
def test_reinserted_points_land_with_their_twins(orc, case):
    """A copy of a build point (same vector and attributes) joins the twin's
    partition and sub-partition: the final assignment is the argmin against
    the final centroids, and Algorithm 1 placed every point in the first
    level whose tag it holds."""
    w = _tiny(80, **case)
    idx = orc.build_from_workload(w, iters=3)
    sel = np.arange(0, w.n, 3)
    lo = w.label_off
    if w.labels is not None:
        lab = [w.labels[lo[i]:lo[i + 1]] for i in sel]
        loff = np.concatenate([[0], np.cumsum([len(v) for v in lab])]).astype(np.int64)
        labs = np.concatenate(lab).astype(np.uint32) if len(lab) else np.zeros(0, np.uint32)
    else:
        loff, labs = None, None
    iy = orc.insert(idx, w.x[sel], None if w.dense is None else w.dense[sel], loff, labs)
    assert np.array_equal(iy.assign[w.n:], idx.assign[sel])
    assert np.array_equal(iy.level[w.n:], idx.level[sel])
    # the layout stays a disjoint cover in (partition, level, id) order
    assert sorted(iy.perm.tolist()) == list(range(w.n + len(sel)))
    assert iy.offs[0] == 0 and iy.offs[-1] == w.n + len(sel) and np.all(np.diff(iy.offs) >= 0)
    # every partition probed: still the filtered brute force over all points
    r = orc.search(iy, w.q, w.con_off, w.con_attr, w.con_val, 9, w.n_partitions)
    bf = orc.bruteforce(iy.x, iy.tk, w.metric, w.q, w.con_off, w.con_attr, w.con_val, 9)
    assert np.array_equal(r.ids, bf.ids)
    assert np.array_equal(r.dist.view(np.uint32), bf.dist.view(np.uint32))


def _aft_properties(idx):
    tk = idx.tk
    n = idx.x.shape[0]
    h = idx.h
    toks = [set(tk.toks[tk.tok_off[i]:tk.tok_off[i + 1]].tolist()) for i in range(n)]
    for p in range(idx.b):
        members = np.nonzero(idx.assign == p)[0]
        rem = set(members.tolist())
        tags = idx.tags[p].tolist()
        assert len(set(t for t in tags if t >= 0)) == len([t for t in tags if t >= 0])
        for j in range(h):
            t = tags[j]
            if t < 0:
                assert not any(toks[i] for i in rem)
                continue
            counts = {}
            for i in rem:
                for tt in toks[i]:
                    counts[tt] = counts.get(tt, 0) + 1
            best = max(counts.values())
            assert counts[t] == best and t == min(k for k, v in counts.items() if v == best)
            pj = {i for i in rem if t in toks[i]}
            assert pj == set(members[idx.level[members] == j].tolist())
            rem -= pj
        assert rem == set(members[idx.level[members] == h].tolist())
        for i in rem:
            assert not any(t in toks[i] for t in tags if t >= 0)


def _csr_properties(idx, dense=None):
    n = idx.x.shape[0]
    perm, offs = idx.perm, idx.offs
    assert sorted(perm.tolist()) == list(range(n))
    assert offs[0] == 0 and offs[-1] == n and np.all(np.diff(offs) >= 0)
    hp = idx.h + 1
    for s in range(idx.b * hp):
        seg = perm[offs[s]:offs[s + 1]]
        assert np.all(idx.assign[seg] == s // hp)
        assert np.all(idx.level[seg] == s % hp)
        # inside a sub-partition: by dense values (attribute 0 first), then id
        keys = [tuple(dense[i]) + (i,) for i in seg] if dense is not None else [(i,) for i in seg]
        assert all(keys[j] < keys[j + 1] for j in range(len(keys) - 1))


@pytest.mark.parametrize("seed,h,lv", [(0, 0, 0), (1, 1, 0), (2, 2, 0), (3, 4, 0), (4, 2, 12),
                                       (5, 4, 30)])
def test_aft_and_csr_properties(orc, seed, h, lv):
    w = _tiny(seed, n=300, d=4, n_q=1, vocabs=(3, 5, 4), label_vocab=lv, b=6, h=h)
    idx = orc.build_from_workload(w, iters=2)
    _aft_properties(idx)
    _csr_properties(idx, w.dense)


# ------------------------------------------------------------- search
def _tokens(w):
    import oracle
    return oracle.workload_tokens(w)


CASES = [
    # seed, metric, vocabs, label_vocab, h, cmin, cmax, integer
    (10, 0, (3, 4), 0, 2, 0, 2, True),
    (11, 0, (3, 4, 6), 0, 4, 1, 3, False),
    (12, 1, (), 20, 4, 1, 3, False),
    (13, 0, (2, 3), 15, 1, 0, 3, True),
    (14, 1, (4,), 0, 0, 0, 1, False),
    (15, 0, (5, 5), 10, 3, 1, 4, False),
]


@pytest.mark.parametrize("case", CASES)
def test_all_partitions_equals_bruteforce(orc, case):
    seed, metric, voc, lv, h, cmin, cmax, integer = case
    w = _tiny(seed, n=400, d=6, n_q=60, vocabs=voc, label_vocab=lv, metric=metric, b=7, h=h,
              cmin=cmin, cmax=cmax, integer=integer)
    idx = orc.build_from_workload(w, iters=3)
    r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=5, m=7)
    bf = orc.bruteforce(w.x, idx.tk, metric, w.q, w.con_off, w.con_attr, w.con_val, 5)
    assert np.array_equal(r.ids, bf.ids)
    assert np.array_equal(r.dist.view(np.uint32), bf.dist.view(np.uint32))
    # every valid point is a survivor when every partition is probed
    assert np.array_equal(r.n_surv, bf.n_cand)


@pytest.mark.parametrize("case", CASES)
def test_bruteforce_matches_fp64(orc, case):
    seed, metric, voc, lv, h, cmin, cmax, integer = case
    w = _tiny(seed, n=400, d=6, n_q=60, vocabs=voc, label_vocab=lv, metric=metric, b=7, h=h,
              cmin=cmin, cmax=cmax, integer=integer)
    tk = _tokens(w)
    bf = orc.bruteforce(w.x, tk, metric, w.q, w.con_off, w.con_attr, w.con_val, 5)
    ids64, d64, nv = ref64.topk64(w.x, w.dense, w.label_off, w.labels, w.dense_vocab,
                                  w.label_vocab, metric, w.q, w.con_off, w.con_attr, w.con_val, 5)
    assert np.array_equal(bf.n_cand, nv)
    d = w.d
    bound = (d + 2) * 2.0 ** -24
    for i in range(w.n_q):
        valid = ids64[i] >= 0
        assert np.array_equal(bf.ids[i] >= 0, valid)
        a = bf.dist[i][valid].astype(np.float64)
        b = d64[i][valid]
        if metric == 0:
            assert np.all(np.abs(a - b) <= bound * np.maximum(b, 1e-30) + 1e-30)
        else:
            # IP: error relative to sum |x_j q_j| (at most |x||q|)
            scale = np.linalg.norm(w.q[i]) * np.max(np.linalg.norm(w.x, axis=1))
            assert np.all(np.abs(a - b) <= bound * scale)
        # ids agree except where FP64 neighbours are within the bound
        for r in range(valid.sum()):
            if bf.ids[i, r] != ids64[i, r]:
                gap = abs(d64[i][r] - d64[i][min(r + 1, valid.sum() - 1)])
                assert gap <= 2 * bound * max(abs(d64[i][r]), 1.0)
        if integer and metric == 0:
            # integer data: the FP32 distances are exact
            assert np.array_equal(bf.ids[i], ids64[i])


def test_returned_ids_satisfy_constraints(orc):
    w = _tiny(20, n=600, d=5, n_q=80, vocabs=(3, 4, 5), label_vocab=25, b=8, h=3, cmin=0,
              cmax=4)
    idx = orc.build_from_workload(w, iters=3)
    for m in (1, 3, 8):
        r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=6, m=m)
        for i in range(w.n_q):
            mask = ref64.valid_mask(w.dense, w.label_off, w.labels,
                                    ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), 3,
                                    w.dense_vocab, w.label_vocab)
            got = r.ids[i][r.ids[i] >= 0]
            assert np.all(mask[got])
            assert r.n_surv[i] <= r.n_cand[i]


def test_single_attribute_exact_rule_is_literal(orc):
    # one dense attribute and one constraint per query: every earlier tag
    # names another value of the same attribute, so the exact rule picks the
    # same single sub-partition as Algorithm 2 read literally
    w = _tiny(30, n=500, d=4, n_q=50, vocabs=(6,), b=5, h=3, cmin=1, cmax=1)
    idx = orc.build_from_workload(w, iters=2)
    a = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=5, m=3, rule=0)
    b = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=5, m=3, rule=1)
    nz = a.masks != 0
    assert np.array_equal(a.masks[nz], b.masks[nz])
    assert np.array_equal(a.ids, b.ids)


def test_unconstrained_full_probe_is_exact_knn(orc):
    rng = np.random.default_rng(40)
    x = rng.integers(0, 16, size=(500, 8)).astype(np.float32)
    q = rng.integers(0, 16, size=(30, 8)).astype(np.float32)
    dense = rng.integers(0, 3, size=(500, 1)).astype(np.uint32)
    idx = orc.build_index(x, dense, [3], None, None, 0, metric=0, b=6, h=1, iters=3, seed=1)
    off = np.zeros(31, dtype=np.int32)
    e = np.zeros(0, dtype=np.int32)
    r = orc.search(idx, q, off, e, e, k=7, m=6)
    d64 = ((x[None].astype(np.float64) - q[:, None]) ** 2).sum(-1)
    ids = np.arange(500)
    for i in range(30):
        order = np.lexsort((ids, d64[i]))[:7]
        assert r.ids[i].tolist() == order.tolist()
    assert np.all(r.n_cand == 500)


def test_h0_is_ivf_postfilter(orc):
    # h = 0: one sub-partition per partition, so the query scans every probed
    # partition whole and filters afterwards (search-then-filter)
    w = _tiny(41, n=500, d=4, n_q=40, vocabs=(3, 3), b=6, h=0, cmin=1, cmax=2)
    idx = orc.build_from_workload(w, iters=2)
    r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=5, m=2)
    sizes = np.bincount(idx.assign, minlength=6)
    for i in range(w.n_q):
        probed = r.probes[i]
        assert r.n_cand[i] == sizes[probed].sum()
        mask = ref64.valid_mask(w.dense, None, None,
                                ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), 2,
                                w.dense_vocab, 0)
        cand = np.nonzero(np.isin(idx.assign, probed) & mask)[0]
        assert r.n_surv[i] == len(cand)
        d64 = ((w.x[cand].astype(np.float64) - w.q[i]) ** 2).sum(-1)
        want = cand[np.lexsort((cand, d64))][:5]
        got = r.ids[i][r.ids[i] >= 0]
        assert np.array_equal(got, want)


def test_routing_probes_nearest_centroids(orc):
    w = _tiny(42, n=400, d=6, n_q=40, vocabs=(3,), b=9, h=1)
    idx = orc.build_from_workload(w, iters=2)
    r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=3, m=4)
    d64 = ((w.q[:, None].astype(np.float64) - idx.centroids[None]) ** 2).sum(-1)
    for i in range(w.n_q):
        assert set(r.probes[i].tolist()) == set(np.argsort(d64[i], kind="stable")[:4].tolist())


def test_contradictory_and_out_of_range_constraints(orc):
    w = _tiny(43, n=200, d=3, n_q=1, vocabs=(3, 4), label_vocab=5, b=3, h=2)
    idx = orc.build_from_workload(w, iters=1)
    q = np.zeros((5, 3), dtype=np.float32)
    # two values of one dense attribute / value outside vocab / attr outside /
    # duplicate constraint (valid) / label and dense together (valid)
    pairs = [[(0, 1), (0, 2)], [(1, 9)], [(7, 0)], [(0, 1), (0, 1)], [(0, 1), (2, 3)]]
    co = np.cumsum([0] + [len(p) for p in pairs]).astype(np.int32)
    ca = np.array([a for p in pairs for a, _ in p], dtype=np.int32)
    cv = np.array([v for p in pairs for _, v in p], dtype=np.int32)
    r = orc.search(idx, q, co, ca, cv, k=4, m=3)
    for i in range(3):
        assert np.all(r.ids[i] == -1) and r.n_cand[i] == 0
        assert np.all(np.isinf(r.dist[i]))
    mask = ref64.valid_mask(w.dense, w.label_off, w.labels, [(0, 1)], 2, w.dense_vocab, 5)
    assert r.n_surv[3] == mask.sum()
    mask = ref64.valid_mask(w.dense, w.label_off, w.labels, [(0, 1), (2, 3)], 2,
                            w.dense_vocab, 5)
    assert r.n_surv[4] == mask.sum()


def test_c1_recall_against_fp64(orc):
    w = synth.make_c1()
    idx = orc.build_from_workload(w)
    r = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=10, m=4)
    ids64, _, nv = ref64.topk64(w.x, w.dense, w.label_off, w.labels, w.dense_vocab,
                                w.label_vocab, 0, w.q, w.con_off, w.con_attr, w.con_val, 10)
    rec = ref64.recall_at_k(r.ids, ids64, nv, 10).mean()
    full = orc.search(idx, w.q, w.con_off, w.con_attr, w.con_val, k=10, m=32)
    assert ref64.recall_at_k(full.ids, ids64, nv, 10).mean() == 1.0
    assert 0.3 < rec <= 1.0


def test_label_index_bruteforce_equals_mask_bruteforce():
    w = _tiny(91, n=3000, d=7, n_q=40, vocabs=(), label_vocab=30, metric=1, cmin=0, cmax=4, max_labels=8)
    inv = ref64.label_index(w.label_off, w.labels, w.n)
    a = ref64.topk64_labels(w.x, inv, 1, w.q, w.con_off, w.con_attr, w.con_val, 10, 0, range(w.n_q))
    b = ref64.topk64(w.x, None, w.label_off, w.labels, [], w.label_vocab, 1, w.q, w.con_off, w.con_attr,
                     w.con_val, 10)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# ---------------------------------------------------------------- learned partitions (Section 5.2)
def test_bliss_assign_hand_worked(orc):
    g = json.load(open(os.path.join(GOLD, "bliss_assign_worked.json")))
    got = orc.bliss_assign(np.array(g["cand"], np.int32), g["b"])
    assert got.tolist() == g["assign"]


def test_bliss_assign_single_candidate_is_identity(orc):
    rng = np.random.default_rng(7)
    cand = rng.integers(0, 9, size=(500, 1)).astype(np.int32)
    assert np.array_equal(orc.bliss_assign(cand, 9), cand[:, 0])


def test_bliss_assign_balances_when_every_bucket_is_a_candidate(orc):
    # every item may go anywhere: least-loaded placement keeps the loads
    # within one of each other after every item (a most-loaded rule, or a
    # dropped load update, would not)
    rng = np.random.default_rng(8)
    b = 7
    cand = np.stack([rng.permutation(b) for _ in range(300)]).astype(np.int32)
    a = orc.bliss_assign(cand, b)
    for n in (1, 10, 57, 300):
        cnt = np.bincount(a[:n], minlength=b)
        assert cnt.max() - cnt.min() <= 1
    assert all(a[i] in cand[i] for i in range(len(a)))


def test_bliss_assign_prefers_the_better_rank_on_ties(orc):
    # two buckets, equal loads before every even item: the even items take
    # their first choice
    cand = np.array([[1, 0], [1, 0], [0, 1], [0, 1]], np.int32)
    assert orc.bliss_assign(cand, 2).tolist() == [1, 0, 0, 1]


def test_build_assigned_pins(orc):
    # a given assignment: centroids are the FP64 means of their points (an
    # empty partition keeps its initial point); the layout is the AFT/CSR of
    # that assignment
    w = synth.make_tiny(31, n=200, d=6, n_q=1, vocabs=(3, 4), b=5, h=2)
    a = (np.arange(w.n) % 4).astype(np.int32)          # partition 4 stays empty
    init = np.array([3, 17, 40, 99, 150], np.int32)
    ix = orc.build_assigned(w.x, w.dense, w.dense_vocab, None, None, 0, a, metric=0, b=5, h=2, seed=0,
                            init=init)
    for c in range(4):
        mean = w.x[a == c].astype(np.float64).mean(axis=0).astype(np.float32)
        assert np.allclose(ix.centroids[c], mean, rtol=0, atol=2e-6 * max(1.0, float(np.abs(mean).max())))
    assert np.array_equal(ix.centroids[4], w.x[150])
    tags, level = orc.aft(a, 5, 2, orc.tokens_of(w.dense, w.dense_vocab, None, None, 0))
    assert np.array_equal(ix.tags, tags) and np.array_equal(ix.level, level)
