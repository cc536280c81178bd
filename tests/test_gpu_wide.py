"""Larger attribute lengths (the paper's appendix: L = 10 and 100 attributes
per item) as label sets wider than 8: the index widens every point's label
slot row to the next power of two (up to 128) and tests membership by a
binary search over the sorted slots.  Build arrays, probes, masks, ids,
distance bits and counters against the oracle; pass bits against Definition
1; insertion and index files on a wide index."""
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


def _check(orc, oi, ix, w, k, m, modes=(0, 2)):
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    pr, mk = ix.probes(w.q, w.con_off, w.con_attr, w.con_val, m)
    assert np.array_equal(pr.cpu().numpy(), r.probes)
    assert np.array_equal(mk.cpu().numpy().view(np.uint32), r.masks)
    for mode in modes:
        ids, dist, nc, ns = (t.cpu().numpy() for t in ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m,
                                                                  mode=mode, counters=True))
        assert np.array_equal(ids, r.ids), (mode, m)
        assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32)), (mode, m)
        assert np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv), (mode, m)


@pytest.mark.parametrize("n_attrs,p,slots", [(10, 0.3, 16), (100, 0.03, 128)])
@pytest.mark.parametrize("prec", ["none", "bf16"])
def test_wide_attribute_sets(caps, orc, n_attrs, p, slots, prec):
    w = synth.make_wide(n_attrs, p, n=6000, n_q=150, n_partitions=12)
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    assert ix.info()["label_slots"] == slots
    g = ix.export()
    for key in ("assign", "level", "perm", "offs", "tags"):
        assert np.array_equal(g[key], getattr(oi, key)), key
    for m in (1, 5, 12):
        _check(orc, oi, ix, w, 10, m)


def test_wide_mixed_sizes_pass_bits_insert_and_files(caps, orc, tmp_path):
    """Label sets of 1..40 labels (64 slots) beside dense attributes."""
    from oracle import ref64
    rng = np.random.default_rng(7)
    w = synth.make_tiny(77, n=4000, d=24, n_q=80, vocabs=(3, 5), label_vocab=300, b=10, h=3, cmin=0, cmax=4,
                        max_labels=40)
    oi = orc.build_from_workload(w, iters=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="fp8")
    assert ix.info()["label_slots"] == 64
    assert np.array_equal(ix.export()["perm"], oi.perm)
    for m in (2, 10):
        _check(orc, oi, ix, w, 10, m)
    h, n = w.aft_height, w.n
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, 4)
    mask = ix.search_debug(w.q, w.con_off, w.con_attr, w.con_val, 10, 4)[4]
    bits = np.unpackbits(mask.cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    for i in range(w.n_q):
        valid = ref64.valid_mask(w.dense, w.label_off, w.labels, ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i),
                                 w.n_dense, w.dense_vocab, w.label_vocab)
        want = np.zeros(n, bool)
        for p, mk in zip(r.probes[i], r.masks[i]):
            for j in range(h + 1):
                if (int(mk) >> j) & 1:
                    lo, hi = oi.offs[p * (h + 1) + j], oi.offs[p * (h + 1) + j + 1]
                    want[lo:hi] = valid[oi.perm[lo:hi]]
        assert np.array_equal(bits[i], want), i
    # insertion of points with up to 64 labels; more is refused
    x_new = rng.normal(size=(300, 24)).astype(np.float32)
    d_new = rng.integers(0, [3, 5], size=(300, 2)).astype(np.uint32)
    sizes = rng.integers(1, 65, size=300)
    lab = [np.sort(rng.choice(300, s, replace=False)).astype(np.uint32) for s in sizes]
    lo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    lb = np.concatenate(lab)
    ix.insert(x_new, d_new, lo, lb)
    oi = orc.insert(oi, x_new, d_new, lo, lb)
    _check(orc, oi, ix, w, 10, 4)
    too = np.arange(65, dtype=np.uint32)
    with pytest.raises(caps.CapsError) as e:
        ix.insert(x_new[:1], d_new[:1], np.array([0, 65], np.int64), too)
    assert e.value.status == -4
    path = str(tmp_path / "wide.caps")
    ix.save(path)
    iy = caps.Index.load(path)
    assert iy.info() == ix.info()
    for mode in (0, 1, 2):
        a = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 10, 4, mode=mode, counters=True)
        b = iy.search(w.q, w.con_off, w.con_attr, w.con_val, 10, 4, mode=mode, counters=True)
        for u, v in zip(a, b):
            assert np.array_equal(u.cpu().numpy().view(np.uint32), v.cpu().numpy().view(np.uint32))
