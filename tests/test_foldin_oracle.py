"""Pins of the oracle's fold-in (frozen C_w, c_k) and held-out likelihood."""
import math

import numpy as np
import pytest

import oracle
import enum_chain
from test_oracle import _chi2_ok


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def tiny_model(K=3, V=3, M=1, alpha=0.6, beta=0.4, seed=1):
    rng = np.random.default_rng(12)
    T = 24
    w = rng.integers(0, V, T).astype(np.uint32)
    d = rng.integers(0, 4, T).astype(np.uint32)
    z = rng.integers(0, K, T).astype(np.int32)
    z[:9] = 0                                  # uneven c_k
    m = oracle.FrozenModel(w, d, z, V, 4, K, M, alpha, beta, seed)
    cwk = np.zeros((V, K), np.int64)
    np.add.at(cwk, (w, z), 1)
    return m, cwk


@pytest.mark.parametrize("words,M,sweeps,learned,LS", [
    ([0, 2], 1, 1, None, 0),
    ([1, 1, 2], 1, 2, None, 0),
    ([0, 2], 2, 2, None, 0),
    ([2, 0], 1, 2, [5, 1, 3], 2),
    ([1, 2, 1], 1, 1, [1, 4, 2], 1),
])
def test_foldin_law_matches_enumeration(words, M, sweeps, learned, LS):
    K = 3
    m, cwk = tiny_model(K=K, M=M)
    states, pi = enum_chain.fold_distribution(words, K, M, m.alpha, m.beta, m.V, cwk, m.ck,
                                              sweeps, learned, LS)
    index = {s: i for i, s in enumerate(states)}
    n = 15000
    L = len(words)
    docptr = np.arange(n + 1, dtype=np.uint64) * L
    allw = np.tile(np.array(words, np.uint32), n)
    weights = None if learned is None else np.tile(np.array(learned, np.uint32), (n, 1))
    z, _ = m.foldin(docptr, allw, np.arange(n, dtype=np.uint32), sweeps, weights, LS)
    counts = np.zeros(len(states))
    for d in range(n):
        counts[index[tuple(int(x) for x in z[d * L:(d + 1) * L])]] += 1
    p = _chi2_ok(counts, pi, n)
    assert p > 1e-4, p


def test_foldin_enumeration_sensitive_to_frozen_ck():
    """The pin can tell a chain that used the document's own counts in c_k."""
    K = 3
    m, cwk = tiny_model(K=K)
    _, right = enum_chain.fold_distribution([0, 2], K, 1, m.alpha, m.beta, m.V, cwk, m.ck, 2)
    _, wrong = enum_chain.fold_distribution([0, 2], K, 1, m.alpha, m.beta, m.V, cwk,
                                            np.zeros(K), 2)
    assert 0.5 * np.abs(right - wrong).sum() > 4 * np.sqrt(len(right) / 15000)


def test_heldout_ll_single_topic_closed_form():
    """K = 1: theta = 1 and phi_w = (L_w + beta) / (T + V beta)."""
    rng = np.random.default_rng(3)
    V, T = 7, 50
    w = rng.integers(0, V, T).astype(np.uint32)
    d = rng.integers(0, 5, T).astype(np.uint32)
    m = oracle.FrozenModel(w, d, np.zeros(T, np.int32), V, 5, 1, 2, 0.5, 0.1)
    Lw = np.bincount(w, minlength=V)
    docptr = np.array([0, 3, 5], np.uint64)
    z = np.zeros(5, np.int32)
    hoptr = np.array([0, 2, 5], np.uint64)
    how = np.array([0, 6, 1, 1, 3], np.uint32)
    got = m.heldout_ll(docptr, z, hoptr, how)
    want = sum(math.log((Lw[x] + 0.1) / (T + V * 0.1)) for x in how)
    assert abs(got - want) < 1e-12 * abs(want)


def test_foldin_is_per_document():
    """A document's result depends only on its own words and request id."""
    m, _ = tiny_model(K=3, M=2)
    words = np.array([0, 1, 2, 2, 1, 0, 0], np.uint32)
    docptr = np.array([0, 3, 7], np.uint64)
    z_all, _ = m.foldin(docptr, words, [11, 12], 3)
    z_one, _ = m.foldin(np.array([0, 4], np.uint64), words[3:], [12], 3)
    assert np.array_equal(z_all[3:], z_one)
