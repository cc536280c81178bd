"""The index build at the benchmark's full size against the oracle.

The SIFT1M-shaped integer corpus (1M x 128, three dense attributes, B = 1024
partitions, AFT height 2).  The oracle's k-means is too slow to run whole at
this size, so it checks the GPU's build in pieces, each exactly:

* Algorithm 1 after the first-level partition: the oracle's AFT and CSR over
  the GPU's final assignment give the GPU's tags, levels, permutation and
  offsets;
* the final assignment: the oracle's argmin against the GPU's final
  centroids, on 100k sampled points;
* every Lloyd iteration it samples: starting from the GPU's centroids after
  i iterations, the oracle's assignment of 100k sampled points equals the
  GPU's, and the oracle's update of 64 sampled clusters (their members in
  ascending id, FP64 sums) equals the GPU's centroids after i + 1
  iterations; the centroids before the first iteration are the points the
  specified init sampler picks.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

N_ASSIGN = 100_000
N_CLUSTERS = 64
ITERS = (0, 1, 4, 9)


@pytest.fixture(scope="module")
def caps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15014_amd as caps
    caps.lib()
    return caps


@pytest.fixture(scope="module")
def c2():
    return synth.make_c2()


def _sample(n, size, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size, replace=False))


def test_c2_layout_matches_oracle(caps, orc, c2):
    w = c2
    ix = caps.Index.from_workload(w)
    g = ix.export()
    ix.close()
    tags, level = orc.aft(g["assign"], w.n_partitions, w.aft_height, orc.workload_tokens(w))
    perm, offs = orc.csr(g["assign"], level, w.n_partitions, w.aft_height, w.dense)
    assert np.array_equal(g["tags"], tags)
    assert np.array_equal(g["level"], level)
    assert np.array_equal(g["perm"], perm)
    assert np.array_equal(g["offs"], offs)
    s = _sample(w.n, N_ASSIGN, 1)
    assert np.array_equal(orc.assign(w.x[s], g["centroids"]), g["assign"][s])


@pytest.mark.parametrize("it", ITERS)
def test_c2_lloyd_iteration_sampled(caps, orc, c2, it):
    w = c2
    a = caps.Index.from_workload(w, kmeans_iters=it)
    ga = a.export()
    a.close()
    b = caps.Index.from_workload(w, kmeans_iters=it + 1)
    gb = b.export()
    b.close()
    if it == 0:
        init = orc.init_ids(w.seed, w.n, w.n_partitions)
        assert np.array_equal(ga["centroids"].view(np.uint32), w.x[init].view(np.uint32))
    s = _sample(w.n, N_ASSIGN, 10 + it)
    assert np.array_equal(orc.assign(w.x[s], ga["centroids"]), ga["assign"][s])
    counts = np.bincount(ga["assign"], minlength=w.n_partitions)
    live = np.flatnonzero(counts > 0)
    cl = np.sort(np.random.default_rng(20 + it).choice(live, N_CLUSTERS, replace=False))
    members = np.isin(ga["assign"], cl)
    upd = orc.update(w.x[members], ga["assign"][members], ga["centroids"])
    assert np.array_equal(upd[cl].view(np.uint32), gb["centroids"][cl].view(np.uint32))
