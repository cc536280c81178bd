"""Dynamic insertions (Table 1 "Dynamic Insertions") on the GPU against the
oracle: after batches of new points are inserted into a built index, its
partitions, levels, CSR layout and search results (every mode, with and
without a low-precision copy, labels and dense attributes) equal the
oracle's insertion into its own index with the same frozen centroids and
tags; a saved and reloaded index keeps them; a failed insertion leaves the
index unchanged."""
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


def _labels(w, sel):
    if w.labels is None:
        return None, None
    lab = [w.labels[w.label_off[i]:w.label_off[i + 1]] for i in sel]
    lo = np.concatenate([[0], np.cumsum([len(v) for v in lab])]).astype(np.int64)
    lb = np.concatenate(lab).astype(np.uint32) if lo[-1] else np.zeros(0, np.uint32)
    return lo, lb


def _check(orc, oi, ix, w_q, co, ca, cv, modes):
    g = ix.export()
    for key in ("assign", "level", "perm", "offs", "tags"):
        assert np.array_equal(g[key], getattr(oi, key)), key
    assert np.array_equal(g["centroids"].view(np.uint32), oi.centroids.view(np.uint32))
    for m in (1, max(1, oi.b // 2), oi.b):
        r = orc.search(oi, w_q, co, ca, cv, 10, m)
        for mode in modes:
            ids, dist, nc, ns = (t.cpu().numpy() for t in ix.search(w_q, co, ca, cv, 10, m, mode=mode, counters=True))
            if mode == 1:   # own routing on the rounded copies: counts compared with every partition probed
                if m == oi.b:
                    assert np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv)
                continue
            assert np.array_equal(ids, r.ids), (mode, m)
            assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32)), (mode, m)
            assert np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv), (mode, m)


CASES = [
    # seed, n, d, vocabs, label_vocab, b, h, metric, prec
    (90, 3000, 16, (3, 5), 0, 9, 2, 0, "bf16"),
    (91, 2500, 24, (4,), 20, 7, 3, 0, "fp8"),
    (92, 2000, 12, (), 15, 6, 2, 1, "none"),
    (93, 4000, 40, (2, 3), 30, 12, 4, 0, "fp16"),
]


@pytest.mark.parametrize("case", CASES)
def test_insert_batches_match_oracle(caps, orc, case):
    seed, n, d, voc, lv, b, h, metric, prec = case
    w = synth.make_tiny(seed, n=n, d=d, n_q=90, vocabs=voc, label_vocab=lv, metric=metric, b=b, h=h, cmin=0, cmax=3,
                        max_labels=8)
    n0 = n * 2 // 3
    base = np.arange(n0)
    lo, lb = _labels(w, base)
    ix = caps.Index.build(w.x[:n0], None if w.dense is None else w.dense[:n0], w.dense_vocab, lo, lb, w.label_vocab,
                          metric=metric, n_partitions=b, kmeans_iters=2, aft_height=h, seed=seed, precision=prec)
    oi = orc.build_index(w.x[:n0], None if w.dense is None else w.dense[:n0], w.dense_vocab, lo, lb, w.label_vocab,
                         metric=metric, b=b, h=h, iters=2, seed=seed)
    modes = (0, 2) if prec == "none" else (0, 1, 2)
    # three batches of uneven size, then one point
    for a, z in ((n0, n0 + 7), (n0 + 7, n0 + 400), (n0 + 400, n - 1), (n - 1, n)):
        sel = np.arange(a, z)
        lo, lb = _labels(w, sel)
        dn = None if w.dense is None else w.dense[sel]
        ix.insert(w.x[sel], dn, lo, lb)
        oi = orc.insert(oi, w.x[sel], dn, lo, lb)
        assert ix.info()["n"] == z
        _check(orc, oi, ix, w.q, w.con_off, w.con_attr, w.con_val, modes)


def test_insert_then_save_load_and_errors(caps, orc, tmp_path):
    w = synth.make_tiny(95, n=2000, d=10, n_q=60, vocabs=(3, 4), label_vocab=12, b=6, h=2, cmin=0, cmax=3)
    n0 = 1500
    lo, lb = _labels(w, np.arange(n0))
    ix = caps.Index.build(w.x[:n0], w.dense[:n0], w.dense_vocab, lo, lb, w.label_vocab, n_partitions=6,
                          kmeans_iters=2, aft_height=2, seed=95, precision="bf16")
    sel = np.arange(n0, 2000)
    lo2, lb2 = _labels(w, sel)
    before = ix.export()
    # a failed insertion (a dense value outside its vocabulary) changes nothing
    bad = w.dense[sel].copy()
    bad[3, 0] = 99
    with pytest.raises(caps.CapsError) as e:
        ix.insert(w.x[sel], bad, lo2, lb2)
    assert e.value.status == -1
    with pytest.raises(caps.CapsError):
        ix.insert(w.x[sel], w.dense[sel], None, None)          # labels missing on a labelled index
    xb = w.x[sel].copy()
    xb[0, 0] = np.nan
    with pytest.raises(caps.CapsError):
        ix.insert(xb, w.dense[sel], lo2, lb2)
    after = ix.export()
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    ix.insert(w.x[sel], w.dense[sel], lo2, lb2)
    path = str(tmp_path / "grown.caps")
    ix.save(path)
    iy = caps.Index.load(path)
    a, b = ix.export(), iy.export()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    for mode in (0, 1, 2):
        x = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 10, 3, mode=mode, counters=True)
        y = iy.search(w.q, w.con_off, w.con_attr, w.con_val, 10, 3, mode=mode, counters=True)
        for u, v in zip(x, y):
            assert np.array_equal(u.cpu().numpy().view(np.uint32), v.cpu().numpy().view(np.uint32))
