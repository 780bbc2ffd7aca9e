"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the NYTimes-shaped corpus (~99M tokens, K=1000, M=2) through init and
one full iteration, every token compared bit for bit after each phase; and a
PubMed-shaped corpus (K=1e4, M=4; 200k documents of the 8M-document shape) for
two iterations.  The oracle computes its own state from the same seeded
inputs (it takes ~4M tokens/s on one core)."""
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
    c = synth.zipf_corpus(200_000, 140_000, 1.05, 90.0, 0.7, synth.CORPUS_SEED_BASE + 2)
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
    """K = 1e6 (the huge-K single-GPU share): V = 1M Zipf(1.1) words, lognormal
    (mean 100, sigma 1) documents, 60k documents of the 20M-document shape.
    Columns longer than one workgroup use hashed global counts; the head word
    (2L > K) uses dense global counts."""
    wl = synth.WORKLOADS["clueweb-share-k1e6"]
    c = synth.zipf_corpus(60_000, 1_000_000, 1.1, 100.0, 1.0, synth.CORPUS_SEED_BASE + 3)
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
