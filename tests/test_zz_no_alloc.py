"""caps_search_static (the search entry point that allocates nothing: its
workspace is the library's static device array) against caps_search: the
same ids, distance bits and counters, on two calls in a row, the second with
a smaller batch; batches large enough to be cut into sub-batches that fit
the static workspace, and small ones; every search mode."""
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
def index(caps):
    w = synth.make_c2(n=60_000, n_q=3000, n_partitions=512)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision="bf16")
    return w, ix


def _sub(w, n):
    sel = np.arange(n)
    co = np.concatenate([[0], np.cumsum(np.diff(w.con_off)[sel])]).astype(np.int32)
    return w.q[:n], co, w.con_attr[:co[-1]], w.con_val[:co[-1]]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_static_equals_allocating_search(caps, index, mode):
    import torch
    w, ix = index
    k, m = 10, 400
    # the first batch needs far more than the 64 MiB static workspace (sub-batches)
    assert ix.workspace_bytes(w.n_q, k, m, mode=mode) > (64 << 20)
    for n in (w.n_q, 700):
        args = _sub(w, n)
        a = ix.search(*args, k, m, mode=mode, counters=True)
        b = ix.search_static(*args, k, m, mode=mode, counters=True)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy().view(np.uint32), y.cpu().numpy().view(np.uint32)), (mode, n)


def test_static_rejects_oversized_budget(caps, index):
    w, ix = index
    with pytest.raises(caps.CapsError) as e:
        ix.search_static(*_sub(w, 10), 10, 8, workspace_bytes=(64 << 20) + 1)
    assert e.value.status == -1
    ids, _ = ix.search_static(*_sub(w, 10), 10, 8, workspace_bytes=1 << 20)   # a smaller budget is fine
    ref, _ = ix.search(*_sub(w, 10), 10, 8)
    assert np.array_equal(ids.cpu().numpy(), ref.cpu().numpy())
