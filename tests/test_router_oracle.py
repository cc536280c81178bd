"""Pins for the router oracle (oracle/router.py): the hash against splitmix64's
published outputs, the backward pass against central finite differences in
FP64, closed forms of the loss, and the Adam step against its definition."""
import os

import numpy as np
import pytest

from oracle import router

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 0x9E3779B97F4A7C15


def test_mix64_is_splitmix64_output_function():
    # splitmix64 emits mix64(seed + i * gamma) for i = 1, 2, ...
    for line in open(os.path.join(GOLD, "splitmix64_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, vals = line.split(":")
        want = [int(v) for v in vals.split()]
        got = [router.mix64(int(seed) + (i + 1) * GAMMA) for i in range(len(want))]
        assert got == want


def _tiny(seed, n=9, d=13, hid=8, b=5):
    rng = np.random.default_rng(seed)
    dp = router.pad_width(d)
    x = np.zeros((n, dp))
    x[:, :d] = rng.normal(size=(n, d))
    x[:, d + rng.integers(0, 64, size=n)] = 1.0
    w1 = rng.normal(size=(hid, dp)) * 0.3
    b1 = rng.normal(size=hid) * 0.1
    w2 = rng.normal(size=(b, hid)) * 0.3
    b2 = rng.normal(size=b) * 0.1
    labels = -np.ones((n, 3), dtype=np.int64)
    for i in range(n):
        k = rng.integers(0, 4)          # 0..3 labels, possibly repeated
        labels[i, :k] = rng.integers(0, b, size=k)
    return x, labels, dict(w1=w1, b1=b1, w2=w2, b2=b2)


def test_backward_matches_central_differences():
    x, labels, p = _tiny(1)
    loss, g = router.loss_and_grads(x, labels, exact=True, **p)
    eps = 1e-6
    for name in ("w1", "b1", "w2", "b2"):
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += eps
            lp, _ = router.loss_and_grads(x, labels, exact=True, **q)
            q[name][idx] -= 2 * eps
            lm, _ = router.loss_and_grads(x, labels, exact=True, **q)
            num[idx] = (lp - lm) / (2 * eps)
        err = np.abs(num - g[name]).max() / max(np.abs(num).max(), 1e-12)
        assert err < 1e-6, (name, err)


def test_uniform_logits_closed_form():
    # W2 = 0, b2 = 0: every logit is 0, softmax is uniform, the loss of a row
    # with labels is log B and its logit gradient (1/B - y) / n
    x, labels, p = _tiny(2, b=7)
    p["w2"][:] = 0.0
    p["b2"][:] = 0.0
    loss, g = router.loss_and_grads(x, labels, exact=True, **p)
    has = (labels >= 0).any(axis=1)
    assert np.isclose(loss, has.sum() * np.log(7) / x.shape[0])
    y = router.label_weights(labels, 7)
    dz = np.where(has[:, None], (1.0 / 7 - y) / x.shape[0], 0.0)
    assert np.allclose(g["b2"], dz.sum(axis=0))


def test_labels_are_sets_and_padding_is_ignored():
    y = router.label_weights(np.array([[2, 2, -1], [-1, -1, -1], [0, 3, 1]]), 4)
    assert np.allclose(y[0], [0, 0, 1, 0]) and not y[1].any()
    assert np.allclose(y[2], [1 / 3, 1 / 3, 0, 1 / 3])


def test_adam_step_definition():
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.5, -0.25])}
    mom = {"w": np.zeros(2)}
    vel = {"w": np.zeros(2)}
    out = router.adam(p, g, mom, vel, 1, 0.1, 0.9, 0.999, 1e-8)
    # first step: bias-corrected moments are g and g^2, so the step is lr * sign(g)
    assert np.allclose(out["w"], p["w"] - 0.1 * np.sign(g["w"]), atol=1e-7)


def test_training_reduces_loss():
    x, labels, p = _tiny(3, n=40, b=6)
    mom = {k: np.zeros_like(v) for k, v in p.items()}
    vel = {k: np.zeros_like(v) for k, v in p.items()}
    l0, _ = router.loss_and_grads(x, labels, **p)
    for step in range(1, 201):
        _, g = router.loss_and_grads(x, labels, **p)
        p = router.adam(p, g, mom, vel, step, 1e-2, 0.9, 0.999, 1e-8)
    l1, _ = router.loss_and_grads(x, labels, **p)
    assert l1 < 0.5 * l0


def test_input_rows_embedding():
    q = np.arange(6, dtype=np.float32).reshape(2, 3)
    # dense vocab (3, 4), labels 5: pairs (0,1) (1,3) (2,4) (0,9 invalid) (5 invalid attr)
    co = np.array([0, 3, 5])
    ca = np.array([0, 1, 2, 0, 5])
    cv = np.array([1, 3, 4, 9, 0])
    x = router.input_rows(q, co, ca, cv, [3, 4], 5, 0.5, -1.0)
    assert x.shape == (2, router.pad_width(3))
    assert np.array_equal(x[:, :3], q * 0.5 - 1.0)
    toks0 = [1, 3 + 3, 7 + 4]          # dense off = (0, 3, 7), label off = 7
    want = np.zeros(64)
    for t in toks0:
        want[router.mix64(t) % 64] = 1.0
    assert np.array_equal(x[0, 3:67], want)
    assert not x[1, 3:].any()          # only invalid pairs
    assert not x[:, 67:].any()         # padding
