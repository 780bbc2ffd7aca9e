"""Encoder oracle (binary64 numpy) -- TEST INFRASTRUCTURE ONLY.

The MLP of the learned fold-in proposal, written out plainly:
  x: bucket b(w) = ((w * 0x9E3779B1 mod 2^32) * buckets) >> 32 of each distinct
     bucket of a document, value count / L (binary32 division);
  a1 = b1 + sum_n x_n W1[b_n];  h1 = relu(a1)
  a2 = h1 W2 + b2;              h2 = relu(a2)
  z  = h2 W3 + b3;              q  = softmax(z)
  loss = -(1/B) sum_b sum_k theta_bk log q_bk
and its gradients by the chain rule.  With round=True the operands of every
matrix product (weights, h1, h2 and the back-propagated signals into a
product) are rounded to bfloat16 (round to nearest even, via binary32) at the
points where the GPU rounds them; with round=False the whole computation is
exact binary64, which is what the finite-difference pin checks.
"""
from __future__ import annotations

import numpy as np


def features(buckets: int, words):
    w = np.asarray(words, dtype=np.uint64)
    b = (((w * 0x9E3779B1) & 0xFFFFFFFF) * buckets) >> 32
    idx, cnt = np.unique(b.astype(np.uint32), return_counts=True)
    val = (cnt.astype(np.float32) / np.float32(len(w))).astype(np.float32)
    return idx, val


def batch_features(buckets, docs):
    rows, idxs, vals = [0], [], []
    for d in docs:
        i, v = features(buckets, d)
        idxs.append(i)
        vals.append(v)
        rows.append(rows[-1] + len(i))
    return np.array(rows, np.uint32), np.concatenate(idxs), np.concatenate(vals)


def bf16(x):
    """Round to bfloat16 (nearest even) through binary32; returns float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward_backward(weights, rowptr, idx, val, theta, round=True):
    """Returns (loss, probs, grads) for a batch; weights = [W1,b1,W2,b2,W3,b3]."""
    R = bf16 if round else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3 = [np.asarray(w, np.float64) for w in weights]
    B = len(rowptr) - 1
    theta = np.asarray(theta, np.float64)
    W1b, W2b, W3b = R(W1), R(W2), R(W3)
    val = np.asarray(val, np.float64)
    a1 = np.tile(b1, (B, 1))
    for b in range(B):
        for n in range(rowptr[b], rowptr[b + 1]):
            a1[b] += val[n] * W1b[idx[n]]
    h1b = R(np.maximum(a1, 0))
    a2 = h1b @ W2b + b2
    h2b = R(np.maximum(a2, 0))
    z = h2b @ W3b + b3
    zmax = z.max(1, keepdims=True)
    lse = zmax + np.log(np.exp(z - zmax).sum(1, keepdims=True))
    logq = z - lse
    q = np.exp(logq)
    loss = -(theta * logq).sum() / B
    g3 = (q - theta) / B
    g3b = R(g3)
    dW3 = h2b.T @ g3b
    db3 = g3.sum(0)
    d2 = g3b @ W3b.T
    g2 = d2 * (a2 > 0)
    g2b = R(g2)
    dW2 = h1b.T @ g2b
    db2 = g2.sum(0)
    d1 = g2b @ W2b.T
    g1 = d1 * (a1 > 0)
    dW1 = np.zeros_like(W1)
    for b in range(B):
        for n in range(rowptr[b], rowptr[b + 1]):
            dW1[idx[n]] += val[n] * g1[b]
    db1 = g1.sum(0)
    return loss, q, [dW1, db1, dW2, db2, dW3, db3]
