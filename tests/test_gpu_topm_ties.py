"""Routing with tied centroid scores (Algorithm 2, top m partitions): the
partitions come in identical pairs (every point of both equal to the pair's
integer centre, so the two centroids and every query's two scores are equal),
and the m-th and the seed probes' s-th best partitions of a query fall inside
tied pairs for odd m and s.  The selection must take ties by ascending
partition id, as the oracle does; searches over the pairs are compared with
the oracle bit for bit."""
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


@pytest.fixture(scope="module")
def paired(caps, orc):
    b, per, d = 256, 4, 16   # 128 pairs of partitions, 4 points each (power-of-two means are exact)
    w = synth.make_tiny(61, n=b * per, d=d, n_q=48, vocabs=(3, 5), b=b, h=2, cmin=0, cmax=2)
    rng = np.random.default_rng(7)
    centres = rng.integers(0, 256, size=(b // 2, d)).astype(np.float32)
    a = np.repeat(np.arange(b, dtype=np.int32), per)
    w.x[:] = centres[a // 2]
    w.q[:] = rng.integers(0, 256, size=w.q.shape).astype(np.float32)
    ix = caps.Index.build(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, metric=w.metric,
                          n_partitions=b, aft_height=2, seed=3, assign=a, precision="bf16")
    oi = orc.build_assigned(w.x, w.dense, w.dense_vocab, w.label_off, w.labels, w.label_vocab, a,
                            metric=w.metric, b=b, h=2, seed=3)
    cent = ix.export()["centroids"]
    assert np.array_equal(cent[0::2].view(np.uint32), cent[1::2].view(np.uint32))   # the pairs tie exactly
    return w, ix, oi


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("m", [33, 64, 153, 201])
def test_tied_partition_scores_match_oracle(paired, orc, mode, m):
    w, ix, oi = paired
    k = 5
    ids, dist, nc, ns = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, counters=True)
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    assert np.array_equal(ids.cpu().numpy(), r.ids)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), r.dist.view(np.uint32))
    assert np.array_equal(nc.cpu().numpy(), r.n_cand)
    assert np.array_equal(ns.cpu().numpy(), r.n_surv)
