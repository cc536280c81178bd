"""GPU parity at the benchmark's full size, on sampled queries.

The workload the benchmark times: the SIFT1M-shaped integer corpus (1M x 128,
three dense attributes, B = 1024 partitions, AFT height 2), 10k filtered
queries searched as one batch at nprobe 624, k = 10, squared L2, on an index
that holds the BF16 copy (search mode 0: matrix-core bounds, exact FP32
rescoring; mode 2: the plain FP32 scan).  The oracle's query path (Alg. 2,
§5.2) runs over the GPU-built partitions for a sample of the queries; ids,
distances, candidate and survivor counts must agree bit for bit.  The search
without counters is the launch configuration the benchmark times; the one
with counters adds the survivor count.  Mode 1 (approximate BF16 keys, FP32
rerank of the best 4k) is checked by its properties: exact filter counts,
valid ids, exact distances, recall against the exact result.
"""
import numpy as np
import pytest

import synth
from oracle import ref64

pytestmark = pytest.mark.gpu

N_SAMPLE = 384
NPROBE = 624
K = 10


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15014_amd as caps
    caps.lib()
    w = synth.make_c2()
    ix = caps.Index.from_workload(w, precision="bf16")
    dev = torch.device("cuda", 0)
    dq = tuple(torch.from_numpy(a).to(dev) for a in (w.q, w.con_off, w.con_attr, w.con_val))
    return w, ix, dq


@pytest.fixture(scope="module")
def sampled(full, orc):
    """Oracle results for a seeded sample of the queries, over the GPU-built index's
    partitions and CSR layout."""
    w, ix, _ = full
    g = ix.export()
    oi = orc.Index(w.x, orc.workload_tokens(w), w.metric, w.n_partitions, w.aft_height, g["centroids"],
                   g["assign"], g["tags"], g["level"], g["perm"], g["offs"], np.zeros(0, np.int32))
    sel = np.sort(np.random.default_rng(2308).choice(w.n_q, N_SAMPLE, replace=False))
    co = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sel])]).astype(np.int32)
    ca = np.concatenate([w.con_attr[w.con_off[i]:w.con_off[i + 1]] for i in sel]).astype(np.int32)
    cv = np.concatenate([w.con_val[w.con_off[i]:w.con_off[i + 1]] for i in sel]).astype(np.int32)
    return sel, orc.search(oi, w.q[sel], co, ca, cv, K, NPROBE), orc.search(oi, w.q[sel], co, ca, cv, 64, NPROBE)


@pytest.mark.parametrize("mode", [0, 2])
def test_full_size_sampled_parity(full, sampled, mode):
    import torch
    w, ix, (q, co, ca, cv) = full
    sel, r, _ = sampled
    dev = q.device
    ids = torch.empty((w.n_q, K), dtype=torch.int32, device=dev)
    dist = torch.empty((w.n_q, K), dtype=torch.float32, device=dev)
    ix.search(q, co, ca, cv, K, NPROBE, mode=mode, out=(ids, dist))
    ids, dist = ids.cpu().numpy()[sel], dist.cpu().numpy()[sel]
    assert np.array_equal(ids, r.ids), mode
    assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32)), mode
    ids2, dist2, nc, ns = ix.search(q, co, ca, cv, K, NPROBE, mode=mode, counters=True)
    assert np.array_equal(ids2.cpu().numpy()[sel], r.ids), mode
    assert np.array_equal(dist2.cpu().numpy()[sel].view(np.uint32), r.dist.view(np.uint32)), mode
    assert np.array_equal(nc.cpu().numpy()[sel], r.n_cand), mode
    assert np.array_equal(ns.cpu().numpy()[sel], r.n_surv), mode
    # the sample exercises the filter: candidates pass the sub-partition
    # lookup and only a fraction of them satisfy the constraints
    assert (r.n_cand > 0).all() and (r.n_surv < r.n_cand).all()


def test_full_size_sampled_mode1(full, sampled):
    w, ix, (q, co, ca, cv) = full
    sel, r, wide = sampled
    ids, dist, nc, ns = ix.search(q, co, ca, cv, K, NPROBE, mode=1, rerank=40, counters=True)
    ids, dist = ids.cpu().numpy()[sel], dist.cpu().numpy()[sel]
    nc, ns = nc.cpu().numpy()[sel], ns.cpu().numpy()[sel]
    # (mode 1 routes with the rounded centroid copy: its probe set may differ
    # from the FP32 routing's near the m-th centroid, so its counts are
    # compared by properties)
    hit = tot = 0
    for j, i in enumerate(sel):
        valid = ids[j] >= 0
        assert valid.sum() == min(K, ns[j])
        mask = ref64.valid_mask(w.dense, w.label_off, w.labels,
                                ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), w.n_dense,
                                w.dense_vocab, w.label_vocab)
        assert np.all(mask[ids[j][valid]])
        exact = {int(a): b for a, b in zip(wide.ids[j], wide.dist[j].view(np.uint32)) if a >= 0}
        for a, b in zip(ids[j][valid], dist[j][valid].view(np.uint32)):
            if int(a) in exact:
                assert exact[int(a)] == b
        t = set(r.ids[j][r.ids[j] >= 0].tolist())
        hit += len(t & set(ids[j][valid].tolist()))
        tot += len(t)
    assert hit / max(tot, 1) >= 0.97, hit / max(tot, 1)


def test_full_size_truth_is_bruteforce(full, orc):
    """The recall truth the benchmark uses (every partition probed) is the
    oracle's filtered brute force (Appendix "Groundtruth") on 256 sampled
    queries: ids, distance bits and |D_C|, in both exact modes."""
    w, ix, (q, co, ca, cv) = full
    sel = np.sort(np.random.default_rng(4).choice(w.n_q, 256, replace=False))
    sco = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sel])]).astype(np.int32)
    sca = np.concatenate([w.con_attr[w.con_off[i]:w.con_off[i + 1]] for i in sel]).astype(np.int32)
    scv = np.concatenate([w.con_val[w.con_off[i]:w.con_off[i + 1]] for i in sel]).astype(np.int32)
    bf = orc.bruteforce(w.x, orc.workload_tokens(w), w.metric, w.q[sel], sco, sca, scv, K)
    for mode in (0, 2):
        ids, dist, nc, ns = ix.search(q, co, ca, cv, K, w.n_partitions, mode=mode, counters=True)
        assert np.array_equal(ids.cpu().numpy()[sel], bf.ids), mode
        assert np.array_equal(dist.cpu().numpy()[sel].view(np.uint32), bf.dist.view(np.uint32)), mode
        assert np.array_equal(ns.cpu().numpy()[sel], bf.n_surv), mode
        assert (nc.cpu().numpy()[sel] <= w.n).all() and (nc.cpu().numpy()[sel] >= bf.n_surv).all(), mode
