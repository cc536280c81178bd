"""Index files: a saved and reloaded index (with its low-precision copy and
its router, Adam state included) answers every query exactly as the
original; damaged files are refused."""
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


def test_save_load_roundtrip(caps, tmp_path):
    w = synth.make_tiny(500, n=3000, d=24, n_q=120, vocabs=(3, 5), label_vocab=25, b=12, h=3, cmin=0, cmax=3)
    ix = caps.Index.from_workload(w, kmeans_iters=3, precision="bf16")
    truth, _ = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 10, 12)
    labels = ix.router_labels(truth)
    ix.router_train(w.q, w.con_off, w.con_attr, w.con_val, labels, hidden=32, epochs=2, batch=64, seed=3,
                    fallback_prob=0.05)
    path = str(tmp_path / "index.caps")
    ix.save(path)
    iy = caps.Index.load(path)
    a, b = ix.export(), iy.export()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    la, lb = ix.export_lowp(), iy.export_lowp()
    for key in ("codes", "scale", "xnorm"):
        assert np.array_equal(la[key], lb[key]), key
    ra, rb = ix.router_get(), iy.router_get()
    for key in ra:
        assert np.array_equal(ra[key], rb[key]), key
    assert ix.router_info() == iy.router_info()
    assert ix.info() == iy.info()
    for mode in (0, 1, 2):
        for routing in (0, 1):
            x = ix.search(w.q, w.con_off, w.con_attr, w.con_val, 7, 5, mode=mode, routing=routing, counters=True)
            y = iy.search(w.q, w.con_off, w.con_attr, w.con_val, 7, 5, mode=mode, routing=routing, counters=True)
            for u, v in zip(x, y):
                assert np.array_equal(u.cpu().numpy().view(np.uint32), v.cpu().numpy().view(np.uint32))
    # continuing training from the loaded Adam state matches continuing the original
    la_ = ix.router_train(w.q, w.con_off, w.con_attr, w.con_val, labels, hidden=32, epochs=1, batch=64, seed=4,
                          reset=0, fallback_prob=0.05)
    lb_ = iy.router_train(w.q, w.con_off, w.con_attr, w.con_val, labels, hidden=32, epochs=1, batch=64, seed=4,
                          reset=0, fallback_prob=0.05)
    assert np.array_equal(la_, lb_)
    ra, rb = ix.router_get(), iy.router_get()
    for key in ra:
        assert np.array_equal(ra[key], rb[key]), key


def test_damaged_files_are_refused(caps, tmp_path):
    w = synth.make_tiny(501, n=800, d=8, n_q=4, vocabs=(3,), b=4, h=1)
    ix = caps.Index.from_workload(w, kmeans_iters=2)
    path = tmp_path / "ok.caps"
    ix.save(str(path))
    raw = path.read_bytes()
    bad = tmp_path / "trunc.caps"
    bad.write_bytes(raw[: len(raw) // 2])
    with pytest.raises(caps.CapsError) as e:
        caps.Index.load(str(bad))
    assert e.value.status == -6
    flip = bytearray(raw)
    flip[8] = 99   # version
    bad.write_bytes(bytes(flip))
    with pytest.raises(caps.CapsError) as e:
        caps.Index.load(str(bad))
    assert e.value.status == -6


def _array_offsets(raw):
    """Byte offset of each array payload of an index file: the header length
    is stored after the magic and version; then (u32 tag, u64 bytes,
    payload) records follow in tag order."""
    hb = int(np.frombuffer(raw[12:16], np.uint32)[0])
    o = 16 + hb
    out = {}
    while o + 12 <= len(raw):
        tag = int(np.frombuffer(raw[o:o + 4], np.uint32)[0])
        nb = int(np.frombuffer(raw[o + 4:o + 12], np.uint64)[0])
        out[tag] = (o + 12, nb)
        o += 12 + nb
        if tag == 16:
            break
    return out


def _refused(caps, path):
    with pytest.raises(caps.CapsError) as e:
        caps.Index.load(str(path))
    assert e.value.status == -6


def test_inconsistent_contents_are_refused(caps, tmp_path):
    """A file whose frame is intact but whose partition layout is damaged
    (an offset, a permutation entry, a tag, the low-precision row width) is
    refused before any search can read through it."""
    w = synth.make_tiny(502, n=900, d=20, n_q=4, vocabs=(3, 4), label_vocab=6, b=5, h=2)
    ix = caps.Index.from_workload(w, kmeans_iters=2, precision="bf16")
    path = tmp_path / "ok.caps"
    ix.save(str(path))
    raw = path.read_bytes()
    caps.Index.load(str(path)).close()
    offs = _array_offsets(raw)
    bad = tmp_path / "bad.caps"

    def patch(tag, index, value, dtype=np.int32):
        b = bytearray(raw)
        at, nb = offs[tag]
        arr = np.frombuffer(bytes(b[at:at + nb]), dtype).copy()
        arr[index] = value
        b[at:at + nb] = arr.tobytes()
        bad.write_bytes(bytes(b))

    patch(4, 3, 10**6)             # offs: a range past the end
    _refused(caps, bad)
    patch(4, 2, -1)                # offs: decreasing
    _refused(caps, bad)
    p0 = np.frombuffer(raw[offs[5][0]:offs[5][0] + 4], np.int32)[0]
    patch(5, 1, p0)                # perm: a repeated id
    _refused(caps, bad)
    patch(5, 0, 900)               # perm: an id out of range
    _refused(caps, bad)
    patch(3, 0, 10**5)             # tags: a token outside the vocabulary
    _refused(caps, bad)
    patch(7, 0, 9, np.int8)        # level: disagrees with the range holding the point
    _refused(caps, bad)
    b = bytearray(raw)             # header: dpad of the BF16 copy doubled
    dp = np.frombuffer(raw[44:48], np.int32)[0]
    assert dp == 32
    b[44:48] = np.int32(64).tobytes()
    bad.write_bytes(bytes(b))
    _refused(caps, bad)
