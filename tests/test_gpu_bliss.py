"""Learned partitions (Section 5.2, CAPS-BLISS) on the GPU against the
oracle: a build from a given first-level assignment lays out exactly the
oracle's (centroids: one update of the initial points with that assignment;
AFT tags, levels, CSR), searches over it equal the oracle's, and one BLISS
round (the router's top-K partitions of every point, the re-partitioning
rule, a rebuild) gives an index whose searches match the oracle's on the
same partitions."""
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


def _pair(caps, orc, w, a, b, h, seed=5):
    ix = caps.Index.build(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, metric=w.metric,
                          n_partitions=b, aft_height=h, seed=seed, assign=a)
    oi = orc.build_assigned(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, a,
                            metric=w.metric, b=b, h=h, seed=seed)
    return ix, oi


def _check(orc, ix, oi, w, ks=(7,), ms=(1, 5, 16)):
    g = ix.export()
    assert np.array_equal(g["assign"], oi.assign)
    assert np.array_equal(g["centroids"].view(np.uint32), oi.centroids.view(np.uint32))
    for key in ("tags", "level", "perm", "offs"):
        assert np.array_equal(g[key], getattr(oi, key)), key
    for k in ks:
        for m in ms:
            ids, dist, nc, ns = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=2, counters=True)
            r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
            assert np.array_equal(ids.cpu().numpy(), r.ids)
            assert np.array_equal(dist.cpu().numpy().view(np.uint32), r.dist.view(np.uint32))
            assert np.array_equal(nc.cpu().numpy(), r.n_cand)
            assert np.array_equal(ns.cpu().numpy(), r.n_surv)


@pytest.mark.parametrize("metric", [0, 1])
def test_assigned_build_matches_oracle(caps, orc, metric):
    w = synth.make_tiny(41, n=3000, d=24, n_q=60, vocabs=(3, 5), label_vocab=12, b=16, h=2, cmin=0, cmax=3,
                        metric=metric)
    a = np.random.default_rng(2).integers(0, 15, size=w.n).astype(np.int32)   # partition 15 stays empty
    ix, oi = _pair(caps, orc, w, a, 16, 2)
    _check(orc, ix, oi, w)


def test_assigned_build_rejects_out_of_range(caps):
    w = synth.make_tiny(42, n=200, d=8, n_q=1, vocabs=(3,), b=4, h=1)
    a = np.zeros(w.n, np.int32)
    a[7] = 4
    with pytest.raises(caps.CapsError):
        caps.Index.build(w.x, w.dense, w.dense_vocab, n_partitions=4, aft_height=1, assign=a)


def test_bliss_round_matches_oracle(caps, orc):
    """Router trained on filtered-neighbour labels, its top-K partitions of
    every point (routing-only probes with the learned router), the
    re-partitioning rule (the library's host call against the oracle's),
    then the rebuild against the oracle's build on the same assignment."""
    w = synth.make_routed(n=20_000, n_q=800, purity=1.0)
    b = w.n_partitions
    ix = caps.Index.from_workload(w)
    truth, _ = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 10, b)
    labels = ix.router_labels(truth)
    ix.router_train(w.q, w.con_off, w.con_attr, w.con_val, labels, hidden=128, epochs=5, batch=256, lr=2e-3,
                    in_scale=1.0 / 3.0, seed=3)
    none_off = np.zeros(w.n + 1, np.int32)
    none = np.zeros(1, np.int32)
    cand, _ = ix.probes(w.x, none_off, none, none, 4, routing=1)
    cand = cand.cpu().numpy()
    a = caps.bliss_assign(cand, b)
    assert np.array_equal(a, orc.bliss_assign(cand, b))
    assert all(a[i] in cand[i] for i in range(0, w.n, 97))
    ix2, oi = _pair(caps, orc, w, a, b, w.aft_height, seed=w.seed)
    _check(orc, ix2, oi, w, ks=(10,), ms=(2, 8))
