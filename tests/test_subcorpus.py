"""The one-column / one-row harness (tests/subcorpus.py) against the whole
oracle: sampled columns and rows of a corpus with long and short columns and
rows, K below and above the longest column, reproduce the whole oracle's word
and doc phases exactly."""
import numpy as np
import pytest

import oracle
import subcorpus as SC
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("K,M", [(50, 2), (3000, 4)])
def test_columns_and_rows_reproduce_the_whole_corpus(K, M):
    rng = np.random.default_rng(K + M)
    V, D = 80, 60
    lens = rng.integers(1, 400, D)
    lens[:2] = 3000
    T = int(lens.sum())
    p = np.arange(1, V + 1, dtype=float) ** -1.1
    words = rng.choice(V, size=T, p=p / p.sum()).astype(np.uint32)
    docs = np.repeat(np.arange(D, dtype=np.uint32), lens)
    perm = rng.permutation(T)
    c = synth.Corpus(words[perm], docs[perm], V, D)
    alpha, beta, seed = 0.1, 0.01, 9
    o = oracle.Oracle(c.word_ids, c.doc_ids, V, D, K, M, alpha, beta, seed=seed)
    o.init()
    o.iterate(1)
    it = o.iteration
    z0, p0 = o.assignments()
    ck0 = o.topic_counts()
    o.word_phase()
    z1, p1 = o.assignments()
    ck1 = o.topic_counts()
    o.doc_phase()
    z2, p2 = o.assignments()
    colstart = np.concatenate([[0], np.cumsum(np.bincount(c.word_ids, minlength=V))])
    rowstart = np.concatenate([[0], np.cumsum(np.bincount(c.doc_ids, minlength=D))])
    for w in [0, 1, 5, 30, 79]:
        idx = SC.column_order(c.word_ids, c.doc_ids, w)
        if len(idx) == 0:
            continue
        zn, pn = SC.column_phase(V, K, M, alpha, beta, seed, it, int(colstart[w]), c.doc_ids[idx],
                                 z0[idx], p0[:, idx], ck0)
        assert np.array_equal(zn, z1[idx]) and np.array_equal(pn, p1[:, idx]), w
    for d in [0, 1, 2, 17, 59]:
        idx = SC.row_order(c.word_ids, c.doc_ids, d)
        zn, pn = SC.row_phase(V, K, M, alpha, beta, seed, it, int(rowstart[d]), c.word_ids[idx],
                              z1[idx], p1[:, idx], ck1)
        assert np.array_equal(zn, z2[idx]) and np.array_equal(pn, p2[:, idx]), d
