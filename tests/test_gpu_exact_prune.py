"""GPU parity of exact search on indexes that hold a low-precision copy.

Search mode 0 then scans the copy with matrix cores to bound every pair's
FP32 distance from below and rescores only the pairs whose bound can beat the
query's current k-th key.  The results must be those of the plain FP32 scan
and of the CPU oracle, bit for bit: ids, distances, candidate and survivor
counts.  Mode 2 forces the plain scan on the same index.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

PRECS = ["bf16", "fp16", "fp8"]


@pytest.fixture(scope="module")
def caps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15014_amd as caps
    caps.lib()
    return caps


def _search(ix, q, co, ca, cv, k, m, mode, rule=0, rescue_grid=0):
    ids, dist, nc, ns = ix.search(q, co, ca, cv, k, m, rule=rule, mode=mode, counters=True, rescue_grid=rescue_grid)
    return ids.cpu().numpy(), dist.cpu().numpy(), nc.cpu().numpy(), ns.cpu().numpy()


def _check(orc, oi, ix, q, co, ca, cv, k, m, rule=0, rescue_grid=0):
    r = orc.search(oi, q, co, ca, cv, k, m, rule=rule)
    for mode in (0, 2):
        ids, dist, nc, ns = _search(ix, q, co, ca, cv, k, m, mode, rule, rescue_grid)
        assert np.array_equal(ids, r.ids), (mode, k, m)
        assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32)), (mode, k, m)
        assert np.array_equal(nc, r.n_cand), (mode, k, m)
        assert np.array_equal(ns, r.n_surv), (mode, k, m)


CASES = [
    # seed, n, d, metric, vocabs, label_vocab, b, h, cmin, cmax, integer
    (200, 900, 5, 0, (3, 4), 0, 7, 2, 0, 2, False),
    (201, 1500, 16, 0, (5, 9, 3), 0, 12, 4, 1, 3, True),
    (202, 900, 12, 1, (), 40, 9, 4, 1, 4, False),
    (203, 1200, 33, 0, (2, 3), 25, 10, 1, 0, 3, False),
    (204, 2000, 64, 0, (4, 4, 4, 4), 60, 16, 3, 0, 5, False),
    (205, 1100, 100, 1, (3,), 0, 6, 2, 0, 1, False),
    (206, 700, 130, 0, (2,), 12, 4, 2, 0, 2, False),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", CASES)
def test_exact_prune_matches_oracle(caps, orc, case, prec):
    seed, n, d, metric, voc, lv, b, h, cmin, cmax, integer = case
    w = synth.make_tiny(seed, n=n, d=d, n_q=130, vocabs=voc, label_vocab=lv, metric=metric, b=b, h=h,
                        cmin=cmin, cmax=cmax, integer=integer, max_labels=8)
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    for m in sorted({1, max(1, b // 3), b}):
        for k in (1, 7, 33):
            _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, 5, max(1, b // 2), rule=1)


@pytest.mark.parametrize("prec", PRECS)
def test_exact_prune_wide_dynamic_range(caps, orc, prec):
    """Points and queries over ten decades, ties, zero vectors and exact
    duplicates of queries: the bound must stay below every exact distance."""
    w = synth.make_tiny(210, n=1600, d=40, n_q=120, vocabs=(3,), label_vocab=0, b=8, h=1, cmin=0, cmax=1)
    rng = np.random.default_rng(210)
    w.x[:: 7] *= np.float32(1e3)
    w.x[3:: 11] *= np.float32(1e-4)
    w.x[5] = 0.0
    w.x[6] = w.x[7]                     # duplicate points: ties broken by id
    w.q[:: 5] *= np.float32(1e2)
    w.q[1:: 9] *= np.float32(1e-3)
    w.q[2] = w.x[100]                   # a query equal to a point (distance 0)
    w.q[3] = 0.0
    w.q[4] = w.x[6]
    w.q += rng.normal(size=w.q.shape).astype(np.float32) * (np.arange(w.n_q) % 3 == 0)[:, None]
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    for m in (1, 3, 8):
        for k in (1, 10, 64):
            _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, k, m)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_exact_prune_c1(caps, orc, prec):
    w = synth.make_c1()
    oi = orc.build_from_workload(w)
    ix = caps.Index.from_workload(w, precision=prec)
    for m in (1, 4, 9, 32):
        _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, 10, m)


def test_exact_prune_integer_corpus(caps, orc):
    """C2-shaped integer vectors (exact in BF16: zero error norms), dense
    filters over three attributes: the tightest bound, most pruning."""
    w = synth.make_c2(n=20_000, n_q=300, n_partitions=64)
    oi = orc.build_from_workload(w, iters=4)
    ix = caps.Index.from_workload(w, kmeans_iters=4, precision="bf16")
    for m in (4, 16, 40, 64):
        _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, 10, m)


def _shell(c):
    """Integer points at squared distance exactly 25 from c: c +- 5 e_i and
    c + (+-3 e_i +- 4 e_j), c + (+-4 e_i +- 3 e_j) for i < j."""
    d = len(c)
    out = []
    for i in range(d):
        for s in (-5, 5):
            v = c.copy()
            v[i] += s
            out.append(v)
    for i in range(d):
        for j in range(i + 1, d):
            for a, b in ((3, 4), (4, 3)):
                for sa in (-1, 1):
                    for sb in (-1, 1):
                        v = c.copy()
                        v[i] += sa * a
                        v[j] += sb * b
                        out.append(v)
    return np.array(out, np.float32)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_exact_prune_equidistant_shell(caps, orc, prec):
    """Four thousand points at exactly the same distance from most queries,
    spread over many partitions: the later probes find far more pairs that
    tie with the seed bound than a query's deferred list holds, so part of
    them is rescored inside the scan.  Ties go to the smaller id."""
    d = 32
    w = synth.make_tiny(220, n=8000, d=d, n_q=40, vocabs=(3,), label_vocab=0, b=64, h=1, cmin=0, cmax=1,
                        integer=True)
    c = np.full(d, 50.0, np.float32)
    sh = _shell(c)
    assert len(sh) == 2 * d + 8 * d * (d - 1) // 2
    rng = np.random.default_rng(220)
    w.x[rng.permutation(w.n)[:len(sh)]] = sh
    w.q[:30] = c
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    for m in (48, 64):
        for k in (10, 64):
            _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    # the rescue pass with a grid of one and of three workgroups: each walks
    # several of the flagged queries' tiles in turn
    for rg in (1, 3):
        _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, 64, 64, rescue_grid=rg)


def test_exact_prune_edge_cases(caps, orc):
    w = synth.make_tiny(17, n=500, d=6, n_q=5, vocabs=(3, 4), label_vocab=10, b=5, h=2)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    q = np.random.default_rng(0).normal(size=(8, 6)).astype(np.float32)
    pairs = [[], [(0, 1), (0, 2)], [(1, 99)], [(9, 0)], [(0, 1), (0, 1)], [(2, 3), (2, 3), (0, 0)],
             [(2, 0), (2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (2, 6), (2, 7), (2, 8)], [(0, -1)]]
    co = np.cumsum([0] + [len(p) for p in pairs]).astype(np.int32)
    ca = np.array([a for p in pairs for a, _ in p], dtype=np.int32)
    cv = np.array([v for p in pairs for _, v in p], dtype=np.int32)
    for k in (1, 64):
        for m in (1, 5):
            _check(orc, oi, ix, q, co, ca, cv, k, m)
    e = ix.search(np.zeros((0, 6), np.float32), np.zeros(1, np.int32), np.zeros(0, np.int32),
                  np.zeros(0, np.int32), 3, 2)
    assert e[0].shape == (0, 3)


def test_exact_prune_batch_invariance(caps):
    w = synth.make_tiny(18, n=3000, d=24, n_q=200, vocabs=(4, 6), label_vocab=30, b=20, h=3, cmin=0,
                        cmax=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision="bf16")
    a = _search(ix, w.q, w.con_off, w.con_attr, w.con_val, 10, 6, 0)
    b = _search(ix, w.q, w.con_off, w.con_attr, w.con_val, 10, 6, 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    rng = np.random.default_rng(3)
    for _ in range(4):
        sub = np.sort(rng.choice(w.n_q, size=rng.integers(1, 70), replace=False))
        co = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sub])]).astype(np.int32)
        ca = np.concatenate([w.con_attr[w.con_off[i]:w.con_off[i + 1]] for i in sub]).astype(np.int32)
        cv = np.concatenate([w.con_val[w.con_off[i]:w.con_off[i + 1]] for i in sub]).astype(np.int32)
        ids, dist = ix.search(w.q[sub], co, ca, cv, 10, 6)
        assert np.array_equal(ids.cpu().numpy(), a[0][sub])
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), a[1][sub].view(np.uint32))


@pytest.mark.parametrize("prec,d", [("bf16", 128), ("fp16", 64), ("bf16", 32)])
def test_chunk_skip_selective_queries_match_oracle(caps, orc, prec, d):
    """Large sub-partitions laid out by attribute values and selective queries
    (2-3 of 3 dense attributes constrained) in batches of several tiles, so
    that the 32 x 32 main pass often skips a row chunk for a wave (no query
    of the wave can pass a row there by the chunk's AND/OR word summary).  Results
    and counters must equal the oracle's bit for bit; the oracle's layout
    has every sub-partition ordered by dense values, then id."""
    w = synth.make_tiny(220 + d, n=24000, d=d, n_q=700, vocabs=(4, 8, 16), label_vocab=0, b=4, h=1,
                        cmin=2, cmax=3, integer=True)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision=prec)
    g = ix.export()
    assert np.array_equal(g["perm"], oi.perm) and np.array_equal(g["offs"], oi.offs)
    for s in range(len(oi.offs) - 1):
        seg = oi.perm[oi.offs[s]:oi.offs[s + 1]]
        keys = [tuple(w.dense[i]) + (i,) for i in seg]
        assert all(keys[j] < keys[j + 1] for j in range(len(keys) - 1))
    for m in (1, 2, 4):
        for k in (1, 10):
            _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    ix.close()
