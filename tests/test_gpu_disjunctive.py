"""Disjunctive constraints on the GPU against the oracle.

A query's constraint list may join AND-terms with OR (pairs with attr ==
CAPS_OR separate the terms; Section 5.3 "Query Algorithm": with OR several
sub-partitions of a partition join the candidate set).  The chosen
sub-partitions are the union of every satisfiable term's choice and a point
is valid when it satisfies some term.  Probes, sub-partition masks, ids,
distance bits, candidate and survivor counts must equal the oracle's; the
per-position pass bits must equal the disjunction of Definition 1 evaluated
on the raw attributes.
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


CASES = [
    # seed, n, d, vocabs, label_vocab, b, h, metric, integer
    (70, 2500, 16, (3, 5, 4), 0, 9, 2, 0, False),
    (71, 2000, 24, (4,), 20, 7, 3, 0, True),
    (72, 1800, 12, (), 15, 6, 2, 1, False),
    (73, 3000, 40, (2, 3), 30, 12, 4, 0, False),
]


def _workload(case, n_q=120):
    seed, n, d, voc, lv, b, h, metric, integer = case
    w = synth.make_tiny(seed, n=n, d=d, n_q=n_q, vocabs=voc, label_vocab=lv, metric=metric, b=b, h=h,
                        integer=integer, max_labels=8)
    rng = np.random.default_rng(seed + 100)
    co, ca, cv = synth.draw_disjunctions(rng, n_q, n, w.dense, w.label_off, w.labels, 1, 4, 0, 2)
    # edge cases in the last rows: an empty term, a contradictory or
    # out-of-range term beside a good one, five terms, only bad terms
    nd = len(voc)
    extra = [[(-1, 0)], [(-1, 0), (-1, 0)]]
    if nd:
        extra += [[(0, 0), (0, 1), (-1, 0), (0, 1)], [(0, 99), (-1, 0), (0, 0)],
                  [(0, 0), (-1, 0), (0, 1), (-1, 0), (0, 0), (-1, 0), (0, 1), (-1, 0), (0, 0)],
                  [(0, 99), (-1, 0), (7, 0)]]
    if lv:
        extra += [[(nd, 0), (-1, 0), (nd, 1), (nd, 2)], [(nd, lv + 3), (-1, 0), (nd, 1)]]
    pairs = [list(zip(ca[co[i]:co[i + 1]].tolist(), cv[co[i]:co[i + 1]].tolist())) for i in range(n_q)]
    pairs[-len(extra):] = extra
    w.con_off = np.cumsum([0] + [len(p) for p in pairs]).astype(np.int32)
    w.con_attr = np.array([a for p in pairs for a, _ in p], np.int32)
    w.con_val = np.array([v for p in pairs for _, v in p], np.int32)
    return w


@pytest.mark.parametrize("prec", ["none", "bf16", "fp8"])
@pytest.mark.parametrize("case", CASES)
def test_disjunctive_search_matches_oracle(caps, orc, case, prec):
    w = _workload(case)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision=prec)
    args = (w.q, w.con_off, w.con_attr, w.con_val)
    for m in (1, max(1, w.n_partitions // 3), w.n_partitions):
        for k in (1, 10):
            r = orc.search(oi, *args, k, m, disjunctive=True)
            pr, mk = ix.probes(*args, m, disjunctive=True)
            assert np.array_equal(pr.cpu().numpy(), r.probes)
            assert np.array_equal(mk.cpu().numpy().view(np.uint32), r.masks)
            for mode in ((0, 2) if prec != "none" else (0,)):
                ids, dist, nc, ns = (t.cpu().numpy() for t in
                                     ix.search(*args, k, m, mode=mode, counters=True, disjunctive=True))
                assert np.array_equal(ids, r.ids), (mode, k, m)
                assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32)), (mode, k, m)
                assert np.array_equal(nc, r.n_cand), (mode, k, m)
                assert np.array_equal(ns, r.n_surv), (mode, k, m)
    if prec != "none":
        # mode 1 (its own routing on the rounded copies): valid ids, as many
        # as its survivors allow
        from oracle import ref64
        m = max(1, w.n_partitions // 2)
        r = orc.search(oi, *args, 10, m, disjunctive=True)
        ids, dist, nc, ns = (t.cpu().numpy() for t in
                             ix.search(*args, 10, m, mode=1, counters=True, disjunctive=True))
        for i in range(w.n_q):
            ok = ids[i] >= 0
            assert ok.sum() == min(10, ns[i])
            valid = ref64.valid_mask_dnf(w.dense, w.label_off, w.labels,
                                         ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), w.n_dense,
                                         w.dense_vocab, w.label_vocab)
            assert valid[ids[i][ok]].all()


@pytest.mark.parametrize("case", CASES[:2])
def test_disjunctive_pass_bits_match_definition(caps, orc, case):
    from oracle import ref64
    w = _workload(case, n_q=50)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    assert np.array_equal(ix.export()["perm"], oi.perm)
    h, n = w.aft_height, w.n
    m = max(1, w.n_partitions // 2)
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, m, disjunctive=True)
    ids, dist, nc, ns, mask = ix.search_debug(w.q, w.con_off, w.con_attr, w.con_val, 10, m, disjunctive=True)
    bits = np.unpackbits(mask.cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    for i in range(w.n_q):
        valid = ref64.valid_mask_dnf(w.dense, w.label_off, w.labels,
                                     ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), w.n_dense,
                                     w.dense_vocab, w.label_vocab)
        want = np.zeros(n, bool)
        for p, mk in zip(r.probes[i], r.masks[i]):
            for j in range(h + 1):
                if (int(mk) >> j) & 1:
                    lo, hi = oi.offs[p * (h + 1) + j], oi.offs[p * (h + 1) + j + 1]
                    want[lo:hi] = valid[oi.perm[lo:hi]]
        assert np.array_equal(bits[i], want), i


def test_separator_without_flag_is_unsatisfiable(caps, orc):
    w = _workload(CASES[0], n_q=60)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    ids, _, nc, ns = (t.cpu().numpy() for t in ix.search(w.q, w.con_off, w.con_attr, w.con_val, 5, 4,
                                                          counters=True))
    has_sep = np.array([(w.con_attr[w.con_off[i]:w.con_off[i + 1]] == -1).any() for i in range(w.n_q)])
    assert has_sep.any()
    assert (ids[has_sep] == -1).all() and (nc[has_sep] == 0).all() and (ns[has_sep] == 0).all()
    oi = orc.build_from_workload(w, iters=2)
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 5, 4)
    assert np.array_equal(ids, r.ids)


def test_disjunctive_server_matches_oracle(caps, orc):
    w = _workload(CASES[1], n_q=150)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, 3, disjunctive=True)
    srv = caps.Server(ix, k=10, nprobe=3, mode=0, max_batch=32, streams=2, max_constraints=16, disjunctive=True)
    try:
        tick = {}
        for i in np.random.default_rng(5).permutation(w.n_q):
            lo, hi = w.con_off[i], w.con_off[i + 1]
            tick[srv.submit(w.q[i], w.con_attr[lo:hi], w.con_val[lo:hi])] = int(i)
        srv.drain(60.0)
        got = {}
        while len(got) < len(tick):
            res = srv.poll()
            assert len(res["tickets"])
            for t, a, b in zip(res["tickets"], res["ids"], res["dist"]):
                got[int(t)] = (a.copy(), b.copy())
    finally:
        srv.close()
    for t, i in tick.items():
        assert np.array_equal(got[t][0], r.ids[i]), i
        assert np.array_equal(got[t][1].view(np.uint32), r.dist[i].view(np.uint32)), i
