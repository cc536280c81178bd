"""GPU parity of the precision mode (search mode 1): low-precision copy,
matrix-core scan with exact filtering, exact FP32 rescoring."""
import numpy as np
import pytest

import synth
from oracle import quant, ref64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def caps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15014_amd as caps
    caps.lib()
    return caps


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_lowp_copy_matches_format_spec(caps, orc, prec):
    w = synth.make_tiny(200, n=900, d=40, n_q=1, vocabs=(3, 4), b=6, h=2)
    w.x[:5] *= 1000.0       # wide dynamic range, includes FP8 saturation of x/s rounding
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision=prec)
    g = ix.export()
    lp = ix.export_lowp()
    xc = w.x[g["perm"]]
    dpad = 64
    if prec == "fp8":
        s, c = quant.fp8_rows(xc)
        assert np.array_equal(lp["scale"].view(np.uint32), s.view(np.uint32))
        assert np.array_equal(lp["codes"], quant.pad_cols(c, dpad))
    else:
        bits = quant.bf16_bits(xc) if prec == "bf16" else quant.f16_bits(xc)
        assert np.array_equal(lp["codes"], quant.pad_cols(bits, dpad))
    assert np.array_equal(lp["xnorm"].view(np.uint32), orc.centroid_norms(xc).view(np.uint32))


def _run(ix, w, k, m, mode, rerank=0):
    ids, dist, nc, ns = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=mode, rerank=rerank,
                                  counters=True)
    return ids.cpu().numpy(), dist.cpu().numpy(), nc.cpu().numpy(), ns.cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_exact_on_small_integer_data(caps, orc, prec):
    # coordinates 0..7: BF16/FP16 hold them exactly and every dot product is
    # exact in FP32, so the approximate ranking is the exact one
    w = synth.make_tiny(201, n=3000, d=64, n_q=120, vocabs=(4, 5, 3), label_vocab=20, b=12, h=2,
                        cmin=0, cmax=3, integer=True)
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    # every partition probed (precision-mode routing, which ranks centroids by
    # their rounded copies, cannot change the probe set)
    m = 12
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 10, m)
    ids, dist, nc, ns = _run(ix, w, 10, m, mode=1)
    assert np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv)
    assert np.array_equal(ids, r.ids)
    assert np.array_equal(dist.view(np.uint32), r.dist.view(np.uint32))


CASES = [
    # seed, metric, vocabs, label_vocab, prec
    (210, 0, (4, 6), 0, "bf16"),
    (211, 0, (3,), 30, "fp8"),
    (212, 1, (), 40, "bf16"),
    (213, 1, (), 40, "fp8"),
    (214, 0, (5, 5), 20, "fp16"),
]


@pytest.mark.parametrize("case", CASES)
def test_lowp_general(caps, orc, case):
    seed, metric, voc, lv, prec = case
    w = synth.make_tiny(seed, n=4000, d=96, n_q=150, vocabs=voc, label_vocab=lv, metric=metric, b=16, h=3,
                        cmin=0, cmax=3, max_labels=8)
    if metric == 1:
        w.x /= np.linalg.norm(w.x, axis=1, keepdims=True)
        w.q /= np.linalg.norm(w.q, axis=1, keepdims=True)
    oi = orc.build_from_workload(w, iters=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    k, R = 10, 40
    # m = B: the probe set is every partition whatever the routing scores,
    # so the filter counts are exactly the oracle's; m = 6: recall only
    for m in (w.n_partitions, 6):
        _general_check(orc, oi, ix, w, k, m, R, prec)


def _general_check(orc, oi, ix, w, k, m, R, prec):
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    wide = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 64, w.n_partitions)
    ids, dist, nc, ns = _run(ix, w, k, m, mode=1, rerank=R)
    full = m == w.n_partitions
    if full:   # the filter is exact in both modes
        assert np.array_equal(nc, r.n_cand) and np.array_equal(ns, r.n_surv)
    hit = tot = 0
    for i in range(w.n_q):
        valid = ids[i] >= 0
        assert valid.sum() == min(k, ns[i])
        mask = ref64.valid_mask(w.dense, w.label_off, w.labels,
                                ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i), w.n_dense,
                                w.dense_vocab, w.label_vocab)
        assert np.all(mask[ids[i][valid]])
        # every returned distance is the exact FP32 distance of its id
        exact = {int(a): b for a, b in zip(wide.ids[i], wide.dist[i].view(np.uint32)) if a >= 0}
        for a, b in zip(ids[i][valid], dist[i][valid].view(np.uint32)):
            if int(a) in exact:
                assert exact[int(a)] == b
        # when every survivor fits in the rescored set the result is exact
        if full and ns[i] <= R:
            assert np.array_equal(ids[i], r.ids[i])
            assert np.array_equal(dist[i].view(np.uint32), r.dist[i].view(np.uint32))
        t = set(r.ids[i][r.ids[i] >= 0].tolist())
        hit += len(t & set(ids[i][valid].tolist()))
        tot += len(t)
    recall = hit / max(tot, 1)
    assert recall >= (0.97 if prec != "fp8" else 0.9) - (0.0 if full else 0.05), (m, recall)


def test_lowp_rejects_index_without_copy(caps):
    w = synth.make_tiny(220, n=300, d=8, n_q=4, vocabs=(3,), b=3, h=1)
    ix = caps.Index.from_workload(w, kmeans_iters=1)
    with pytest.raises(caps.CapsError):
        ix.search(w.q, w.con_off, w.con_attr, w.con_val, 5, 2, mode=1)
    ix2 = caps.Index.from_workload(w, kmeans_iters=1, precision="bf16")
    with pytest.raises(caps.CapsError):
        ix2.search(w.q, w.con_off, w.con_attr, w.con_val, 5, 2, mode=1, rerank=3)


def _decoded(rows, prec):
    """FP64 values of the rows' copies in the published formats (and the
    per-row FP8 scale), from the format definitions of oracle/quant.py."""
    rows = np.asarray(rows, np.float32)
    if prec == "bf16":
        return quant.bf16_value(quant.bf16_bits(rows)).astype(np.float64)
    if prec == "fp16":
        return quant.f16_bits(rows).view(np.float16).astype(np.float64)
    s, c = quant.fp8_rows(rows)
    return s[:, None].astype(np.float64) * quant.e4m3_value(c).astype(np.float64)


@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_lowp_routing_scores(caps, orc, prec, metric):
    """Precision-mode routing (the centroid score GEMM on the matrix cores):
    each probe set equals the best m under the score computed from the
    rounded query and centroid copies (FP64 sum of their exact products),
    except for centroids whose scores lie within the FP32 accumulation bound
    of the m-th; and it keeps most of the FP32 probes."""
    w = synth.make_tiny(240 + metric, n=6000, d=40, n_q=200, vocabs=(3,), label_vocab=0, metric=metric, b=64, h=1)
    if metric == 1:
        w.x /= np.linalg.norm(w.x, axis=1, keepdims=True)
        w.q /= np.linalg.norm(w.q, axis=1, keepdims=True)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision=prec)
    cent = ix.export()["centroids"]
    qv, cv = _decoded(w.q, prec), _decoded(cent, prec)
    dot = qv @ cv.T
    cn = orc.centroid_norms(cent).astype(np.float64)
    ref = cn[None, :] - 2 * dot if metric == 0 else -dot
    dpad = 64
    gam = 8 * dpad * 2.0 ** -24
    mag = np.linalg.norm(qv, axis=1)[:, None] * np.linalg.norm(cv, axis=1)[None, :]
    tol = (2 if metric == 0 else 1) * gam * mag + 8 * 2.0 ** -24 * (np.abs(cn)[None, :] + 2 * np.abs(dot)) + 1e-30
    m = 8
    pr, _ = ix.probes(w.q, w.con_off, w.con_attr, w.con_val, m, mode=1)
    p0, _ = ix.probes(w.q, w.con_off, w.con_attr, w.con_val, m, mode=0)
    pr, p0 = pr.cpu().numpy(), p0.cpu().numpy()
    kept = 0
    for i in range(w.n_q):
        order = np.lexsort((np.arange(64), ref[i]))
        want = set(order[:m].tolist())
        got = set(pr[i].tolist())
        assert len(got) == m
        t = ref[i][order[m - 1]]
        for c in got ^ want:
            assert abs(ref[i][c] - t) <= 2 * tol[i].max(), (i, c)
        kept += len(got & set(p0[i].tolist()))
    assert kept / (m * w.n_q) >= 0.9, kept / (m * w.n_q)
