"""GPU parity: libcaps (through its C ABI) against the CPU oracle.

Same seeded inputs on both sides.  Integer work (assignments, levels, CSR,
tags, probes, sub-partition masks, ids, counters) must be bit-exact, and in
FP32 mode the distances too: both sides evaluate the same sequential fma
chains.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def caps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15014_amd as caps
    caps.lib()
    return caps


def _gpu_search(ix, w, k, m, rule=0, q=None):
    q = w.q if q is None else q
    ids, dist, nc, ns = ix.search(q, w.con_off, w.con_attr, w.con_val, k, m, rule=rule, counters=True)
    return ids.cpu().numpy(), dist.cpu().numpy(), nc.cpu().numpy(), ns.cpu().numpy()


def _check_build(orc_idx, g):
    assert np.array_equal(g["centroids"].view(np.uint32), orc_idx.centroids.view(np.uint32))
    assert np.array_equal(g["assign"], orc_idx.assign)
    assert np.array_equal(g["level"], orc_idx.level)
    assert np.array_equal(g["tags"], orc_idx.tags)
    assert np.array_equal(g["offs"], orc_idx.offs)
    assert np.array_equal(g["perm"], orc_idx.perm)


def _check_search(orc, orc_idx, ix, w, k, m, rule=0):
    r = orc.search(orc_idx, w.q, w.con_off, w.con_attr, w.con_val, k, m, rule=rule)
    ids, dist, nc, ns = _gpu_search(ix, w, k, m, rule)
    pr, mk = ix.probes(w.q, w.con_off, w.con_attr, w.con_val, m, rule=rule)
    assert np.array_equal(pr.cpu().numpy(), r.probes)
    assert np.array_equal(mk.cpu().numpy().view(np.uint32), r.masks)
    assert np.array_equal(nc, r.n_cand)
    assert np.array_equal(ns, r.n_surv)
    assert np.array_equal(ids, r.ids)
    assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32))


def test_c1_build_and_search(caps, orc):
    w = synth.make_c1()
    oi = orc.build_from_workload(w)
    ix = caps.Index.from_workload(w)
    _check_build(oi, ix.export())
    for m in (1, 4, 9, 32):
        _check_search(orc, oi, ix, w, 10, m)
    bf = orc.bruteforce(w.x, oi.tk, 0, w.q, w.con_off, w.con_attr, w.con_val, 10)
    ids, dist, _, ns = _gpu_search(ix, w, 10, 32)
    assert np.array_equal(ids, bf.ids)
    assert np.array_equal(ns, bf.n_cand)


CASES = [
    # seed, n, d, metric, vocabs, label_vocab, b, h, cmin, cmax, integer
    (100, 700, 5, 0, (3, 4), 0, 7, 2, 0, 2, False),
    (101, 1500, 16, 0, (5, 9, 3), 0, 12, 4, 1, 3, True),
    (102, 900, 12, 1, (), 40, 9, 4, 1, 4, False),
    (103, 1200, 33, 0, (2, 3), 25, 10, 1, 0, 3, False),
    (104, 600, 8, 1, (6,), 0, 5, 0, 0, 1, False),
    (105, 2000, 64, 0, (4, 4, 4, 4), 60, 16, 3, 0, 5, False),
    (106, 300, 3, 0, (3,), 0, 1, 2, 0, 1, True),
]


@pytest.mark.parametrize("case", CASES)
def test_tiny_parity(caps, orc, case):
    seed, n, d, metric, voc, lv, b, h, cmin, cmax, integer = case
    w = synth.make_tiny(seed, n=n, d=d, n_q=150, vocabs=voc, label_vocab=lv, metric=metric, b=b, h=h,
                        cmin=cmin, cmax=cmax, integer=integer, max_labels=8)
    oi = orc.build_from_workload(w, iters=4)
    ix = caps.Index.from_workload(w, kmeans_iters=4)
    _check_build(oi, ix.export())
    for m in sorted({1, max(1, b // 3), b}):
        for k in (1, 7):
            _check_search(orc, oi, ix, w, k, m)
    _check_search(orc, oi, ix, w, 5, max(1, b // 2), rule=1)


def test_edge_cases(caps, orc):
    import torch
    w = synth.make_tiny(7, n=500, d=6, n_q=5, vocabs=(3, 4), label_vocab=10, b=5, h=2)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2)
    q = np.random.default_rng(0).normal(size=(8, 6)).astype(np.float32)
    pairs = [[], [(0, 1), (0, 2)], [(1, 99)], [(9, 0)], [(0, 1), (0, 1)], [(2, 3), (2, 3), (0, 0)],
             [(2, 0), (2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (2, 6), (2, 7), (2, 8)], [(0, -1)]]
    co = np.cumsum([0] + [len(p) for p in pairs]).astype(np.int32)
    ca = np.array([a for p in pairs for a, _ in p], dtype=np.int32)
    cv = np.array([v for p in pairs for _, v in p], dtype=np.int32)
    r = orc.search(oi, q, co, ca, cv, 64, 5)
    ids, dist, nc, ns = ix.search(q, co, ca, cv, 64, 5, counters=True)
    assert np.array_equal(ids.cpu().numpy(), r.ids)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), r.dist.view(np.uint32))
    assert np.array_equal(nc.cpu().numpy(), r.n_cand)
    # empty batch
    e = ix.search(np.zeros((0, 6), np.float32), np.zeros(1, np.int32), np.zeros(0, np.int32),
                  np.zeros(0, np.int32), 3, 2)
    assert e[0].shape == (0, 3)
    # malformed offsets: the query is unsatisfiable, the others unaffected
    bad = co.copy()
    bad[2] = 10_000
    ids2, _ = ix.search(q, bad, ca, cv, 64, 5)
    ids2 = ids2.cpu().numpy()
    assert np.all(ids2[1] == -1) and np.all(ids2[2] == -1)
    assert np.array_equal(ids2[0], r.ids[0])
    # argument errors
    with pytest.raises(caps.CapsError):
        ix.search(q, co, ca, cv, 0, 2)
    with pytest.raises(caps.CapsError):
        ix.search(q, co, ca, cv, 3, 6)
    torch.cuda.synchronize()


def test_determinism_and_batch_invariance(caps, orc):
    w = synth.make_tiny(8, n=3000, d=24, n_q=200, vocabs=(4, 6), label_vocab=30, b=20, h=3, cmin=0,
                        cmax=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3)
    a = _gpu_search(ix, w, 10, 6)
    b = _gpu_search(ix, w, 10, 6)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    rng = np.random.default_rng(1)
    for _ in range(5):
        sub = np.sort(rng.choice(w.n_q, size=rng.integers(1, 40), replace=False))
        co = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sub])]).astype(np.int32)
        ca = np.concatenate([w.con_attr[w.con_off[i]:w.con_off[i + 1]] for i in sub]).astype(np.int32)
        cv = np.concatenate([w.con_val[w.con_off[i]:w.con_off[i + 1]] for i in sub]).astype(np.int32)
        ids, dist = ix.search(w.q[sub], co, ca, cv, 10, 6)
        assert np.array_equal(ids.cpu().numpy(), a[0][sub])
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), a[1][sub].view(np.uint32))


def test_build_errors(caps):
    x = np.zeros((10, 4), np.float32)
    with pytest.raises(caps.CapsError):
        caps.Index.build(x, n_partitions=11)
    x[3, 1] = np.nan
    with pytest.raises(caps.CapsError):
        caps.Index.build(x, n_partitions=2)
    x = np.zeros((10, 4), np.float32)
    with pytest.raises(caps.CapsError):
        caps.Index.build(x, np.full((10, 1), 5, np.uint32), [3], n_partitions=2)
    lo = np.array([0, 2] + [2] * 9, np.int64)
    with pytest.raises(caps.CapsError):
        caps.Index.build(x, None, None, lo, np.array([1, 1], np.uint32), 4, n_partitions=2)


@pytest.mark.parametrize("b", [200, 700, 2100])
def test_many_partitions(caps, orc, b):
    """Best-m selection over 256 to 4096 sort slots (pb = 256, 1024, 4096):
    probes in the oracle's order (score, then partition id), masks, ids."""
    w = synth.make_tiny(300 + b, n=max(6000, 4 * b), d=6, n_q=60, vocabs=(3, 5), label_vocab=0, b=b, h=2,
                        cmin=0, cmax=2, integer=True)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2)
    _check_build(oi, ix.export())
    for m in (1, 37, b):
        _check_search(orc, oi, ix, w, 10, m)


@pytest.mark.parametrize("prec,mode", [("bf16", 0), ("bf16", 1), ("bf16", 2), ("fp8", 0), ("none", 0)])
def test_sub_batches_equal_one_batch(caps, orc, prec, mode):
    """A workspace budget that splits the batch into several sub-batches (and
    several probe rounds each) gives every query the same ids, distances and
    counters as one batch, and in the exact modes the oracle's results."""
    w = synth.make_tiny(230, n=2500, d=48, n_q=301, vocabs=(4, 6), label_vocab=30, b=40, h=2,
                        cmin=0, cmax=3, max_labels=8)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    m, k = 34, 9   # m >= 32: seed round and main round

    def run(budget):
        ids, dist, nc, ns = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, counters=True,
                                      workspace_bytes=budget)
        return ids.cpu().numpy(), dist.cpu().numpy(), nc.cpu().numpy(), ns.cpu().numpy()

    one = run(0)
    for budget in (40_000, 150_000):   # a few queries per sub-batch; tens of them
        split = run(budget)
        assert np.array_equal(split[0], one[0]), budget
        assert np.array_equal(split[1].view(np.uint32), one[1].view(np.uint32)), budget
        assert np.array_equal(split[2], one[2]), budget
        assert np.array_equal(split[3], one[3]), budget
    if mode != 1:
        oi = orc.build_from_workload(w, iters=3)
        r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
        assert np.array_equal(one[0], r.ids)
        assert np.array_equal(one[1].view(np.uint32), r.dist.view(np.uint32))
        assert np.array_equal(one[2], r.n_cand)
        assert np.array_equal(one[3], r.n_surv)


def test_8192_partitions(caps, orc):
    """The largest supported B: the register top-m network of 32 keys per
    thread (probes query, sorted) and the search's selection at B = 8192."""
    w = synth.make_tiny(8192, n=20_000, d=8, n_q=48, vocabs=(4, 3), label_vocab=0, b=8192, h=1, cmin=0, cmax=2)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2)
    _check_build(oi, ix.export())
    for m in (1, 37, 4097, 8192):
        _check_search(orc, oi, ix, w, 10, m)


def test_nonfinite_queries(caps, orc):
    """A query row holding NaN or Inf has an empty answer on the asynchronous
    path and makes the validating call fail with EINVAL; the other rows are
    unaffected."""
    w = synth.make_tiny(31, n=3000, d=12, n_q=40, vocabs=(3, 5), label_vocab=0, b=8, h=2, cmin=0, cmax=2)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 5, 4)
    q = w.q.copy()
    q[3, 1] = np.nan
    q[7, 0] = np.inf
    q[8, 11] = -np.inf
    bad = np.zeros(w.n_q, bool)
    bad[[3, 7, 8]] = True
    for mode in (0, 1, 2):
        ids, dist = ix.search(q, w.con_off, w.con_attr, w.con_val, 5, 4, mode=mode)
        ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
        assert (ids[bad] == -1).all() and np.isposinf(dist[bad]).all()
        if mode != 1:
            assert np.array_equal(ids[~bad], r.ids[~bad])
            assert np.array_equal(dist[~bad].view(np.uint32), r.dist[~bad].view(np.uint32))
        with pytest.raises(caps.CapsError) as e:
            ix.search(q, w.con_off, w.con_attr, w.con_val, 5, 4, mode=mode, validate=True)
        assert e.value.status == -1
    ids, dist = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 5, 4, validate=True)
    assert np.array_equal(ids.cpu().numpy(), r.ids)
    with pytest.raises(caps.CapsError) as e:
        ix.search_debug(q, w.con_off, w.con_attr, w.con_val, 5, 4)
    assert e.value.status == -1


@pytest.mark.parametrize("case", [
    # seed, n, d, vocabs, label_vocab, b, h, cmin, cmax, mode
    (40, 2500, 16, (3, 5), 0, 9, 2, 0, 3, 0),
    (41, 2500, 16, (3, 5), 30, 9, 3, 0, 4, 2),
    (42, 1800, 40, (), 25, 6, 4, 1, 4, 0),
])
def test_survivor_mask_matches_definition(caps, orc, case):
    """Per CSR position, the filter's pass bit for every (query, chosen
    sub-partition): equal to Definition 1 evaluated on the raw attributes
    over the sub-partitions the oracle chose, and summing to the survivor
    count."""
    from oracle import ref64
    seed, n, d, voc, lv, b, h, cmin, cmax, mode = case
    w = synth.make_tiny(seed, n=n, d=d, n_q=60, vocabs=voc, label_vocab=lv, b=b, h=h, cmin=cmin, cmax=cmax,
                        max_labels=8)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    assert np.array_equal(ix.export()["perm"], oi.perm)   # the same CSR positions on both sides
    m = max(1, b // 2)
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, m)
    ids, dist, nc, ns, mask = ix.search_debug(w.q, w.con_off, w.con_attr, w.con_val, 10, m, mode=mode)
    assert np.array_equal(ids.cpu().numpy(), r.ids)
    assert np.array_equal(ns.cpu().numpy(), r.n_surv)
    bits = np.unpackbits(mask.cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    for i in range(w.n_q):
        valid = ref64.valid_mask(w.dense, w.label_off, w.labels,
                                 ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), w.n_dense,
                                 w.dense_vocab, w.label_vocab)
        want = np.zeros(n, bool)
        for p, mk in zip(r.probes[i], r.masks[i]):
            for j in range(h + 1):
                if (int(mk) >> j) & 1:
                    lo, hi = oi.offs[p * (h + 1) + j], oi.offs[p * (h + 1) + j + 1]
                    want[lo:hi] = valid[oi.perm[lo:hi]]
        assert np.array_equal(bits[i], want), i
        assert bits[i].sum() == r.n_surv[i]


def test_height_sweep(caps, orc):
    """The ablation's AFT heights h in {0, 1, 2, 4, 8} on a C2-shaped
    corpus: each index equals the oracle's (Algorithm 1 for that h) and
    answers as the oracle; with the exact sub-partition rule the answers at
    a given nprobe are the same for every h while the candidates scanned
    shrink."""
    w = synth.make_c2(n=30_000, n_q=300, n_partitions=64)
    base = orc.build_from_workload(w, iters=3, h=0)
    tk = base.tk
    prev_nc, ref = None, {}
    for h in (0, 1, 2, 4, 8):
        tags, level = orc.aft(base.assign, w.n_partitions, h, tk)
        perm, offs = orc.csr(base.assign, level, w.n_partitions, h, w.dense)
        oi = orc.Index(base.x, tk, 0, w.n_partitions, h, base.centroids, base.assign, tags, level, perm, offs,
                       base.init)
        ix = caps.Index.from_workload(w, kmeans_iters=3, aft_height=h, precision="bf16")
        _check_build(oi, ix.export())
        for m in (8, 32):
            r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, m)
            ids, dist, nc, ns = _gpu_search(ix, w, 10, m)
            assert np.array_equal(ids, r.ids) and np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv)
            assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32))
            if m in ref:
                assert np.array_equal(ids, ref[m])
            else:
                ref[m] = ids
            if m == 32:
                if prev_nc is not None:
                    assert (nc <= prev_nc).all()
                prev_nc = nc
        ix.close()


@pytest.mark.parametrize("mode,prec", [(0, "bf16"), (1, "bf16"), (2, "none"), (0, "none")])
def test_workspace_exact_fit(caps, orc, mode, prec):
    """A search given exactly the workspace the library reports for the
    batch, or one byte less (then cut into sub-batches), equals the search
    with the default budget.  Each sub-batch's allocation is the size of a
    dry run of its own carve, and the carve's arena refuses any byte past the
    allocation, so a size formula that missed an array fails here as an
    error instead of overrunning.  (An earlier size formula missed one
    bucketing array and the kernels wrote past the allocation.)"""
    w = synth.make_tiny(61, n=5000, d=40, n_q=300, vocabs=(3, 7), label_vocab=10, b=48, h=3, cmin=0, cmax=3)
    ix = caps.Index.from_workload(w, precision=prec)
    for k, m in ((1, 1), (10, 12), (64, 48)):
        need = ix.workspace_bytes(w.n_q, k, m, mode=mode)
        a = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, counters=True)
        b = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, counters=True, workspace_bytes=need)
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy().view(np.uint32), y.cpu().numpy().view(np.uint32))
        # one byte less: the batch is cut into sub-batches, same results
        c = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, counters=True,
                      workspace_bytes=need - 1)
        for x, y in zip(a, c):
            assert np.array_equal(x.cpu().numpy().view(np.uint32), y.cpu().numpy().view(np.uint32))
