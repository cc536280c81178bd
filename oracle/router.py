"""Learned router: FP64 reference forward, loss, backward and Adam step
(TEST INFRASTRUCTURE ONLY; callers: the test suite).

The router replaces centroid routing by a two-layer perceptron on the query
vector and its constraints (the paper's CAPS-BLISS variant, Section 5.2,
trains partitions on filtered-neighbour labels; here the k-means partitions
stay fixed and only the routing is learned):

    x  = [ q * scale + shift  ||  e(C) ]           input row, zero padded
    h  = relu(W1 x + b1)                             hidden (H)
    z  = W2 h + b2                                   one logit per partition (B)

e(C) is a 64-wide multi-hot vector: each valid constraint pair becomes its
token (dense attribute i, value v: off_i + v; label l: off_L + l) and sets
position mix64(token) mod 64, mix64 being the output function of splitmix64.

Training target: the set S of partitions holding a query's exact filtered
top-k ids; loss = -(1/|S|) sum_{s in S} log softmax(z)_s, averaged over the
batch rows (a row with empty S contributes nothing).  The GPU computes the
matrix products with BF16 operands and FP32 accumulation; `forward` and
`loss_and_grads` take the same BF16 roundings of the operands (weights, the
input row, the hidden activations, the logit and hidden gradients) and do
the arithmetic in FP64.  `exact=True` skips every rounding: that is the
smooth function the finite-difference pins differentiate.
"""
from __future__ import annotations

import numpy as np

from . import quant

M64 = (1 << 64) - 1
EMBED = 64


def mix64(z: int) -> int:
    """splitmix64's output function (Steele, Lea & Flood)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def pad_width(d: int) -> int:
    return (d + EMBED + 31) // 32 * 32


def constraint_tokens(con_off, con_attr, con_val, dense_vocab, label_vocab):
    """Tokens of the valid constraint pairs of every query (a list of lists)."""
    n_dense = len(dense_vocab)
    off = np.concatenate([[0], np.cumsum(np.asarray(dense_vocab, dtype=np.int64))])
    out = []
    for i in range(len(con_off) - 1):
        toks = []
        for e in range(int(con_off[i]), int(con_off[i + 1])):
            a, v = int(con_attr[e]), int(con_val[e])
            if 0 <= a < n_dense and 0 <= v < dense_vocab[a]:
                toks.append(int(off[a]) + v)
            elif a == n_dense and label_vocab > 0 and 0 <= v < label_vocab:
                toks.append(int(off[-1]) + v)
        out.append(toks)
    return out


def input_rows(q, con_off, con_attr, con_val, dense_vocab, label_vocab, scale, shift, exact=False):
    """Input rows [q * scale + shift || e(C) || 0], FP64 values of the BF16
    rows the GPU builds (the affine map evaluated in FP32: product, then sum)."""
    q = np.asarray(q, dtype=np.float32)
    n, d = q.shape
    dp = pad_width(d)
    x = np.zeros((n, dp), dtype=np.float64)
    if exact:
        x[:, :d] = q.astype(np.float64) * scale + shift
    else:
        v = (q * np.float32(scale)).astype(np.float32) + np.float32(shift)
        x[:, :d] = quant.bf16_value(quant.bf16_bits(v.astype(np.float32)))
    for i, toks in enumerate(constraint_tokens(con_off, con_attr, con_val, dense_vocab, label_vocab)):
        for t in toks:
            x[i, d + (mix64(t) % EMBED)] = 1.0
    return x


def _bf(a, exact):
    if exact:
        return np.asarray(a, dtype=np.float64)
    return quant.bf16_value(quant.bf16_bits(np.asarray(a, dtype=np.float32))).astype(np.float64)


def forward(x, w1, b1, w2, b2, exact=False):
    """Logits (n x B) and the hidden activations used by the second layer."""
    hp = x @ _bf(w1, exact).T + np.asarray(b1, dtype=np.float64)
    h = np.maximum(hp, 0.0)
    hb = _bf(h, exact)
    z = hb @ _bf(w2, exact).T + np.asarray(b2, dtype=np.float64)
    return z, hb


def label_weights(labels, b):
    """Rows of the target distribution: uniform over each row's distinct
    labels (entries < 0 are padding)."""
    labels = np.asarray(labels)
    y = np.zeros((labels.shape[0], b), dtype=np.float64)
    for i, row in enumerate(labels):
        s = sorted({int(v) for v in row if v >= 0})
        for v in s:
            y[i, v] = 1.0 / len(s)
    return y


def loss_and_grads(x, labels, w1, b1, w2, b2, exact=False):
    """Mean loss over the batch and the gradients of every parameter."""
    n = x.shape[0]
    b = np.asarray(w2).shape[0]
    z, hb = forward(x, w1, b1, w2, b2, exact)
    y = label_weights(labels, b)
    has = y.sum(axis=1) > 0
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    lse = np.log(ez.sum(axis=1, keepdims=True)) + zmax
    p = ez / ez.sum(axis=1, keepdims=True)
    loss = float(np.sum(np.where(has, (lse[:, 0] * y.sum(axis=1)) - (y * z).sum(axis=1), 0.0)) / n)
    dz = np.where(has[:, None], (p - y) / n, 0.0)
    dzb = _bf(dz, exact)
    gw2 = dzb.T @ hb
    gb2 = dz.sum(axis=0)
    dh = (dzb @ _bf(w2, exact)) * (hb > 0)
    gb1 = dh.sum(axis=0)
    gw1 = _bf(dh, exact).T @ x
    return loss, dict(w1=gw1, b1=gb1, w2=gw2, b2=gb2)


def adam(params, grads, mom, vel, step, lr, beta1, beta2, eps):
    """One Adam step (bias-corrected) on every parameter; step counts from 1."""
    out = {}
    for k in params:
        g = np.asarray(grads[k], dtype=np.float64)
        mom[k] = beta1 * mom[k] + (1.0 - beta1) * g
        vel[k] = beta2 * vel[k] + (1.0 - beta2) * g * g
        mh = mom[k] / (1.0 - beta1 ** step)
        vh = vel[k] / (1.0 - beta2 ** step)
        out[k] = np.asarray(params[k], dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return out
