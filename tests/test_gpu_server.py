"""Serving loop (caps_server_*): results of every request equal, bit for bit,
the same query searched alone and in one batch, whatever mix and timing it
arrives in; admission refuses beyond the queue; the workspace budget caps the
batch; statistics add up."""
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
def work(caps):
    w = synth.make_tiny(400, n=6000, d=40, n_q=400, vocabs=(4, 6), label_vocab=30, b=24, h=2, cmin=0, cmax=3)
    ix = caps.Index.from_workload(w, kmeans_iters=4, precision="bf16")
    return w, ix


def _pairs(w, i):
    lo, hi = w.con_off[i], w.con_off[i + 1]
    return w.con_attr[lo:hi], w.con_val[lo:hi]


def _collect(srv, n_expect):
    got = {}
    srv.drain(60.0)
    while len(got) < n_expect:
        r = srv.poll()
        assert len(r["tickets"]), "results missing after drain"
        for t, a, b, s in zip(r["tickets"], r["ids"], r["dist"], r["status"]):
            assert s == 0
            got[int(t)] = (a.copy(), b.copy())
    return got


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_alone_and_mixed_results_are_identical(caps, work, mode):
    w, ix = work
    k, m = 10, 6
    batch_ids, batch_dist = (t.cpu().numpy() for t in ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m,
                                                                   mode=mode))
    alone = {}
    for i in range(0, w.n_q, 37):
        a, b = ix.search(w.q[i:i + 1], np.array([0, w.con_off[i + 1] - w.con_off[i]], np.int32), *_pairs(w, i),
                         k, m, mode=mode)
        alone[i] = (a.cpu().numpy()[0], b.cpu().numpy()[0])
        assert np.array_equal(alone[i][0], batch_ids[i])
        assert np.array_equal(alone[i][1].view(np.uint32), batch_dist[i].view(np.uint32))
    rng = np.random.default_rng(mode)
    srv = caps.Server(ix, k=k, nprobe=m, mode=mode, max_batch=64, streams=3, batch_window_us=50.0)
    try:
        # one burst in random order, then a Poisson replay of a random subset
        order = rng.permutation(w.n_q)
        tick = {}
        for i in order:
            tick[srv.submit(w.q[i], *_pairs(w, i))] = int(i)
        sub = np.sort(rng.choice(w.n_q, size=150, replace=False))
        co = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sub])]).astype(np.int32)
        ca = np.concatenate([_pairs(w, i)[0] for i in sub]).astype(np.int32)
        cv = np.concatenate([_pairs(w, i)[1] for i in sub]).astype(np.int32)
        arr = np.cumsum(rng.exponential(1.0 / 20_000.0, size=len(sub)))
        tks = srv.replay(w.q[sub], co, ca, cv, arr)
        for t, i in zip(tks, sub):
            assert t != 0
            tick[int(t)] = int(i)
        got = _collect(srv, len(tick))
        for t, i in tick.items():
            ids, dist = got[t]
            assert np.array_equal(ids, batch_ids[i]), (mode, i)
            assert np.array_equal(dist.view(np.uint32), batch_dist[i].view(np.uint32)), (mode, i)
        st = srv.stats()
        assert st["completed"] == st["submitted"] == len(tick) and st["failed"] == 0
        assert st["batches"] >= 1 and 1.0 <= st["mean_batch"] <= 64.0
        assert 0.0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    finally:
        srv.close()


def test_small_polls_between_submits(caps, work):
    """Results taken a few at a time while requests keep arriving (the queues
    are consumed from their heads and compacted as they go): every request
    comes back exactly once, equal bit for bit to the one-batch search."""
    w, ix = work
    k, m = 10, 6
    batch_ids, batch_dist = (t.cpu().numpy() for t in ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m))
    srv = caps.Server(ix, k=k, nprobe=m, max_batch=16, streams=2)
    try:
        tick, got = {}, {}

        def take(r):
            for t, a, b, s in zip(r["tickets"], r["ids"], r["dist"], r["status"]):
                assert s == 0 and int(t) not in got
                got[int(t)] = (a.copy(), b.copy())

        for rep in range(3):
            for i in range(w.n_q):
                tick[srv.submit(w.q[i], *_pairs(w, i))] = i
                if i % 5 == 4:
                    take(srv.poll(7))
        srv.drain(60.0)
        while True:
            r = srv.poll(7)
            if not len(r["tickets"]):
                break
            take(r)
        assert set(got) == set(tick)
        for t, i in tick.items():
            assert np.array_equal(got[t][0], batch_ids[i]), i
            assert np.array_equal(got[t][1].view(np.uint32), batch_dist[i].view(np.uint32)), i
        st = srv.stats()
        assert st["completed"] == st["submitted"] == len(tick) and st["failed"] == 0
    finally:
        srv.close()


def test_queue_full_refuses_and_accepted_requests_finish(caps, work):
    w, ix = work
    srv = caps.Server(ix, k=5, nprobe=24, max_batch=1, streams=1, queue_slots=2)
    try:
        n = 300
        tks = srv.replay(w.q[:n], w.con_off[:n + 1], w.con_attr, w.con_val, np.zeros(n))
        accepted = int((tks != 0).sum())
        st = srv.stats()
        assert st["rejected"] == n - accepted and st["rejected"] > 0
        got = _collect(srv, accepted)
        assert set(got) == {int(t) for t in tks if t != 0}
        with pytest.raises(caps.CapsError):   # more constraints than the server takes
            srv.submit(w.q[0], np.zeros(17, np.int32), np.zeros(17, np.int32))
    finally:
        srv.close()


def test_workspace_budget_caps_the_batch(caps, work):
    w, ix = work
    small = caps.Server(ix, k=10, nprobe=8, max_batch=4096, workspace_bytes=3 << 20)
    try:
        cap = small.stats()["max_batch"]
        assert 1 <= cap < 4096
        for i in range(200):
            small.submit(w.q[i], *_pairs(w, i))
        got = _collect(small, 200)
        assert len(got) == 200
        assert small.stats()["mean_batch"] <= cap
    finally:
        small.close()
    with pytest.raises(caps.CapsError):
        caps.Server(ix, k=10, nprobe=8, workspace_bytes=16)
    with pytest.raises(caps.CapsError):
        caps.Server(ix, k=0, nprobe=8)
    with pytest.raises(caps.CapsError):
        caps.Server(ix, k=10, nprobe=8, routing=1)   # no router on this index


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_server_results_match_oracle(caps, work, orc, mode):
    """Every request served in a mix (random order, three streams, uneven
    batches) against the oracle's Algorithm 2 on its own index: modes 0 and 2
    bit-exact; mode 1 (BF16 routing and scores, FP32 rerank) by its
    properties: only valid ids, as many as its survivors allow, exact FP32
    distances, and recall against the exact answer."""
    from oracle import ref64
    w, ix = work
    oi = orc.build_from_workload(w, iters=4)
    assert np.array_equal(ix.export()["perm"], oi.perm)
    k, m = 10, 6
    r = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, k, m)
    wide = orc.search(oi, w.q, w.con_off, w.con_attr, w.con_val, 64, w.n_partitions)
    # mode 1 routes with the rounded centroid copy: its own filter counts
    ns1 = ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m, mode=1, counters=True)[3].cpu().numpy()
    rng = np.random.default_rng(100 + mode)
    srv = caps.Server(ix, k=k, nprobe=m, mode=mode, max_batch=48, streams=3)
    try:
        tick = {}
        for i in rng.permutation(w.n_q):
            tick[srv.submit(w.q[i], *_pairs(w, i))] = int(i)
        got = _collect(srv, len(tick))
    finally:
        srv.close()
    hit = tot = 0
    for t, i in tick.items():
        ids, dist = got[t]
        if mode != 1:
            assert np.array_equal(ids, r.ids[i]), (mode, i)
            assert np.array_equal(dist.view(np.uint32), r.dist[i].view(np.uint32)), (mode, i)
            continue
        valid = ids >= 0
        assert valid.sum() == min(k, ns1[i])
        mask = ref64.valid_mask(w.dense, w.label_off, w.labels, ref64.pairs_of(w.con_off, w.con_attr, w.con_val, i),
                                w.n_dense, w.dense_vocab, w.label_vocab)
        assert mask[ids[valid]].all()
        exact = {int(a): b for a, b in zip(wide.ids[i], wide.dist[i].view(np.uint32)) if a >= 0}
        for a, b in zip(ids[valid], dist[valid].view(np.uint32)):
            if int(a) in exact:
                assert exact[int(a)] == b
        truth = set(r.ids[i][r.ids[i] >= 0].tolist())
        hit += len(truth & set(ids[valid].tolist()))
        tot += len(truth)
    if mode == 1:
        assert hit / max(tot, 1) >= 0.9, hit / max(tot, 1)


def test_server_shares_workspace_budget(caps, work):
    """The workspace budget is shared by the batches in flight: with room for
    about two batches of 32, three streams still serve everything, batches
    stay within the cap and results equal the one-batch search."""
    w, ix = work
    k, m = 10, 6
    ws32 = ix.workspace_bytes(32, k, m)
    assert ix.workspace_bytes(1, k, m) < ws32 < ix.workspace_bytes(64, k, m)
    budget = ws32 * 5 // 2
    batch_ids, batch_dist = (t.cpu().numpy() for t in ix.search(w.q, w.con_off, w.con_attr, w.con_val, k, m))
    srv = caps.Server(ix, k=k, nprobe=m, mode=0, max_batch=32, streams=3, workspace_bytes=budget)
    try:
        tick = {}
        for i in range(w.n_q):
            tick[srv.submit(w.q[i], *_pairs(w, i))] = i
        got = _collect(srv, len(tick))
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == w.n_q and st["failed"] == 0
    assert st["mean_batch"] <= 32
    for t, i in tick.items():
        assert np.array_equal(got[t][0], batch_ids[i])
        assert np.array_equal(got[t][1].view(np.uint32), batch_dist[i].view(np.uint32))
