"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the NYTimes-shaped corpus (~99M tokens, K=1000, M=2) through init and
one full iteration, every token compared bit for bit after each phase; and a
PubMed-shaped corpus (K=1e4, M=4; 200k documents of the 8M-document shape) for
two iterations, and the first 120k documents of the ClueWeb-shaped share
(K=1e6).  The oracle computes its own state from the same seeded
inputs (it takes ~4M tokens/s on one core).  The PubMed-shaped workload at its
full 8M-document size is checked by properties that hold at any size."""
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


def compare_csc(s, o, where):
    zs, ps = s.assignments(csc=True)
    zo, po = o.csc()
    bad = np.count_nonzero(zs != zo)
    badp = np.count_nonzero(ps != po)
    assert bad == 0 and badp == 0, (where, bad, badp)
    assert np.array_equal(s.topic_counts(), o.topic_counts()), where


@pytest.mark.timeout(900)
def test_nytimes_shape_full_size_iteration(W):
    wl = synth.WORKLOADS["nytimes-shape-k1e3"]
    c = wl.make()
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    s.init()
    o.init()
    compare_csc(s, o, "init")
    s.word_phase()
    o.word_phase()
    compare_csc(s, o, "word phase 1")
    assert s.accepted(1) == o.accepted(1)
    s.doc_phase()
    o.doc_phase()
    compare_csc(s, o, "doc phase 1")
    assert s.accepted(2) == o.accepted(2)
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= 1e-6 * abs(ll_o), (ll_s, ll_o)


@pytest.mark.timeout(900)
def test_pubmed_shape_k1e4_m4(W):
    wl = synth.WORKLOADS["pubmed-shape-k1e4"]
    c = wl.make(200_000)               # the first 200k documents of the full corpus
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    s.init()
    o.init()
    for it in range(2):
        s.word_phase()
        o.word_phase()
        compare_csc(s, o, f"word phase {it + 1}")
        s.doc_phase()
        o.doc_phase()
        compare_csc(s, o, f"doc phase {it + 1}")
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= 1e-6 * abs(ll_o), (ll_s, ll_o)


@pytest.mark.timeout(900)
def test_clueweb_shape_k1e6(W):
    """K = 1e6 (the huge-K single-GPU share): the first 120k documents of the
    ClueWeb-shaped share (V = 1M Zipf(1.1) words, lognormal(mean 100, sigma 1)
    documents; 12M tokens).  Its head word has ~1.5M tokens, more than K, so
    its word proposals take the inverse CDF through prefix counts in global
    memory; shorter long columns use hashed global counts."""
    wl = synth.WORKLOADS["clueweb-share-k1e6"]
    c = wl.make(120_000)
    assert np.bincount(c.word_ids, minlength=c.V).max() > wl.K
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    s.init()
    o.init()
    for it in range(2):
        s.word_phase()
        o.word_phase()
        compare_csc(s, o, f"word phase {it + 1}")
        s.doc_phase()
        o.doc_phase()
        compare_csc(s, o, f"doc phase {it + 1}")
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= 1e-6 * abs(ll_o), (ll_s, ll_o)


@pytest.mark.timeout(900)
def test_pubmed_shape_full_size_properties(W):
    """The PubMed-shaped workload at its full size (8M documents, ~720M
    tokens, K = 1e4, M = 4), in the launch configuration the benchmark uses,
    where the oracle would take hours: checked by properties that hold at any
    size.  Every topic and pending proposal lies in [0, K); the sampler's c_k
    is the exact histogram of its Z and sums to T; acceptance counts are in
    range; the log likelihood is finite and rises over the first iterations;
    and an iteration replayed from a saved state reproduces every token (no
    race or order dependence at full occupancy)."""
    import sys
    wl = synth.WORKLOADS["pubmed-shape-k1e4"]
    log = lambda m: print(f"[pubmed full size] {m}", file=sys.__stderr__, flush=True)
    c = wl.make()
    T, K, M = c.T, wl.K, wl.M
    log(f"corpus T={T}")
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, wl.alpha, wl.beta, seed=3)
    del c
    s.init()
    ll0 = s.log_likelihood()
    s.iterate(1)
    blob = s.save_state()
    s.iterate(1)
    acc_w, acc_d = s.accepted(1), s.accepted(2)
    z, p = s.assignments()
    ck = s.topic_counts()
    ll2 = s.log_likelihood()
    log(f"two iterations, LL {ll0:.6e} -> {ll2:.6e}")
    assert z.min() >= 0 and z.max() < K
    assert p.min() >= 0 and p.max() < K
    assert ck.sum() == T
    assert np.array_equal(ck, np.bincount(z, minlength=K))
    assert 0 < acc_w <= M * T and 0 < acc_d <= M * T
    assert np.isfinite(ll0) and np.isfinite(ll2) and ll2 > ll0
    p_sample = p[:, ::101].copy()
    del p
    s.load_state(blob)
    del blob
    s.iterate(1)
    z2, p2 = s.assignments()
    assert np.array_equal(z, z2)
    assert np.array_equal(p_sample, p2[:, ::101])
    assert np.array_equal(ck, s.topic_counts())
    assert (s.accepted(1), s.accepted(2)) == (acc_w, acc_d)
    log("replay from the saved state matches")
    s.close()


def sampled_check(W, wl, c, M, seed, ranks, row_bins, tag):
    """Bit-exact word phase of sampled columns (the words of the given
    frequency ranks and six short ones) and doc phase of sampled rows (the
    longest and three of each length class), recomputed by the oracle one
    column or row at a time from the sampler's own phase-start state and c_k
    (tests/subcorpus.py)."""
    import sys
    import subcorpus as SC
    log = lambda m: print(f"[{tag}] {m}", file=sys.__stderr__, flush=True)
    K, V = wl.K, c.V
    counts = np.bincount(c.word_ids, minlength=V)
    colstart = np.concatenate([[0], np.cumsum(counts)])
    order = np.argsort(counts)[::-1]
    rng = np.random.default_rng(11)
    words = [int(order[r]) for r in ranks]
    words += [int(w) for w in rng.choice(np.nonzero((counts > 0) & (counts <= 2048))[0], 6, replace=False)]
    sel = np.nonzero(np.isin(c.word_ids, words))[0]
    cols = {w: sel[c.word_ids[sel] == w] for w in words}
    for w, idx in cols.items():
        assert np.all(np.diff(c.doc_ids[idx].astype(np.int64)) >= 0)  # input order is column order
    lens = np.bincount(c.doc_ids, minlength=c.D)
    docs = [int(np.argmax(lens))]
    for lo, hi in row_bins:
        cand = np.nonzero((lens >= lo) & (lens <= hi))[0]
        docs += [int(d) for d in rng.choice(cand, min(3, len(cand)), replace=False)]
    rowstart = {}
    rows = {}
    for d in docs:
        a = int(np.searchsorted(c.doc_ids, d, side="left"))
        b = int(np.searchsorted(c.doc_ids, d, side="right"))
        rowstart[d] = a
        rows[d] = a + np.lexsort((np.arange(b - a), c.word_ids[a:b]))
    log(f"columns {[len(v) for v in cols.values()]}, rows {[len(v) for v in rows.values()]}")

    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, wl.alpha, wl.beta, seed=seed)
    s.init()
    s.iterate(1)
    it = s.iteration

    def take(z, p, sets):
        return {k: (z[v].copy(), p[:, v].copy()) for k, v in sets.items()}

    z, p = s.assignments()
    ck0 = s.topic_counts()
    col_pre = take(z, p, cols)
    del z, p
    s.word_phase()
    z, p = s.assignments()
    ck1 = s.topic_counts()
    col_post, row_pre = take(z, p, cols), take(z, p, rows)
    del z, p
    s.doc_phase()
    z, p = s.assignments()
    row_post = take(z, p, rows)
    del z, p
    s.close()
    log("sampler done; oracle columns")
    for w in words:
        idx = cols[w]
        zn, pn = SC.column_phase(V, K, M, wl.alpha, wl.beta, seed, it, int(colstart[w]), c.doc_ids[idx],
                                 col_pre[w][0], col_pre[w][1], ck0)
        assert np.array_equal(zn, col_post[w][0]), ("column", w, len(idx))
        assert np.array_equal(pn, col_post[w][1]), ("column proposals", w, len(idx))
    log("oracle rows")
    for d in docs:
        idx = rows[d]
        zn, pn = SC.row_phase(V, K, M, wl.alpha, wl.beta, seed, it, rowstart[d], c.word_ids[idx],
                              row_pre[d][0], row_pre[d][1], ck1)
        assert np.array_equal(zn, row_post[d][0]), ("row", d, len(idx))
        assert np.array_equal(pn, row_post[d][1]), ("row proposals", d, len(idx))
    log("all sampled columns and rows match")


@pytest.mark.timeout(900)
def test_pubmed_shape_full_size_sampled_columns_and_rows(W):
    """The PubMed-shaped workload at its full size (8M documents, 720M tokens,
    K = 1e4, M = 4), in the benchmark's launch configuration, bit for bit on
    sampled outputs: columns of every length class (segment kernels and the
    long path up to ~7M tokens, inverse CDF included) and rows of every length
    class (the longest, on the doc long path, included)."""
    wl = synth.WORKLOADS["pubmed-shape-k1e4"]
    c = wl.make()
    sampled_check(W, wl, c, wl.M, 3, (9, 60, 400, 2000),
                  ((1, 64), (65, 128), (129, 256), (257, 1024), (1025, 2048)), "pubmed sampled")


@pytest.mark.timeout(900)
def test_clueweb_share_2m_docs_sampled_columns_and_rows(W):
    """The ClueWeb-shaped share's first 2M documents (200M tokens, V = 1M,
    K = 1e6, M = 2), the slice the benchmark times: sampled columns (~5M
    tokens down to segment sizes; long ones take the inverse CDF through
    global prefix counts and their guide) and rows, bit for bit."""
    wl = synth.WORKLOADS["clueweb-share-k1e6"]
    c = wl.make(2_000_000)
    sampled_check(W, wl, c, wl.M, 3, (4, 30, 300, 3000),
                  ((1, 128), (129, 256), (257, 512), (513, 2048), (2049, 4096)), "clueweb sampled")
