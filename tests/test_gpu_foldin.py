"""Fold-in on the GPU against the oracle: bit-exact assignments (plain and
learned proposal), held-out likelihood within 1e-9 relative, and per-document
results independent of the batch a document is folded in with."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def trained(K=50, M=2, seed=3):
    c = synth.lda_corpus(300, 400, 8, 80.0, 0.5, 0.05, seed)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, 50.0 / K, 0.01, seed=1)
    o.init()
    o.iterate(5)
    z, _ = o.assignments()
    return c, z


def new_docs(V, n, seed, lo=1, hi=3000):
    rng = np.random.default_rng(seed)
    lens = np.clip(rng.lognormal(np.log(120), 1.0, n).astype(int), lo, hi)
    lens[0] = 1
    lens[1] = hi
    docptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    words = rng.integers(0, V, int(docptr[-1])).astype(np.uint32)
    return docptr, words


def synthetic_weights(n, K, seed):
    rng = np.random.default_rng(seed)
    p = rng.dirichlet(np.full(K, 0.3), size=n)
    return (1 + np.floor(p * (1 << 20))).astype(np.uint32)


@pytest.mark.parametrize("learned", [False, True])
def test_foldin_bit_exact(W, learned):
    K, M = 50, 2
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    om = oracle.FrozenModel(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    docptr, words = new_docs(c.V, 60, 5)
    req = np.arange(1000, 1060, dtype=np.uint32)
    wts = synthetic_weights(60, K, 9) if learned else None
    rng = np.random.default_rng(2)
    ho_lens = rng.integers(0, 40, 60)
    hoptr = np.concatenate([[0], np.cumsum(ho_lens)]).astype(np.uint64)
    how = rng.integers(0, c.V, int(hoptr[-1])).astype(np.uint32)
    for sweeps in (1, 4):
        zg, hg = gm.foldin(docptr, words, req, sweeps, wts, 2 if learned else 0, hoptr, how)
        zo, _ = om.foldin(docptr, words, req, sweeps, wts, 2 if learned else 0)
        assert np.array_equal(zg, zo), (learned, sweeps, np.nonzero(zg != zo)[0][:5])
        for d in range(60):
            sl = slice(int(docptr[d]), int(docptr[d + 1]))
            hs = slice(int(hoptr[d]), int(hoptr[d + 1]))
            ho = om.heldout_ll(np.array([0, sl.stop - sl.start], np.uint64), zo[sl],
                               np.array([0, hs.stop - hs.start], np.uint64), how[hs])
            assert abs(hg[d] - ho) <= 1e-9 * max(1.0, abs(ho)), (d, hg[d], ho)


def test_foldin_alone_equals_in_mix(W):
    K, M = 50, 2
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    docptr, words = new_docs(c.V, 30, 8)
    req = np.arange(30, dtype=np.uint32) * 7 + 3
    wts = synthetic_weights(30, K, 4)
    for w in (None, wts):
        zmix, _ = gm.foldin(docptr, words, req, 3, w, 2)
        for d in (0, 1, 17, 29):
            sl = slice(int(docptr[d]), int(docptr[d + 1]))
            zone, _ = gm.foldin(np.array([0, sl.stop - sl.start], np.uint64), words[sl],
                                req[d:d + 1], 3, None if w is None else w[d:d + 1], 2)
            assert np.array_equal(zone, zmix[sl])
