"""The synthetic workloads have the shapes the paper prints in Table 3."""
import json
import os

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
T3 = json.load(open(os.path.join(HERE, "golden", "table3_datasets.json")))


def test_nytimes_shape_matches_table3():
    c = synth.WORKLOADS["nytimes-shape-k1e3"].make()
    ny = T3["NYTimes"]
    assert c.D == ny["D"]
    assert abs(c.T - ny["T"]) <= 0.02 * ny["T"]
    assert abs(c.T / c.D - ny["T_over_D"]) <= 0.02 * ny["T_over_D"]
    assert abs(c.V - ny["V"]) <= 0.03 * ny["V"]
    # every rank of the vocabulary is reachable; the head follows Zipf(1)
    f = np.sort(np.bincount(c.word_ids, minlength=c.V))[::-1]
    assert 8.0 < f[0] / f[9] < 12.0


def test_pubmed_and_clueweb_parameters_match_table3():
    # generating 730M / 2B tokens is a GPU-box job; the parameters are checked here
    pm = T3["PubMed"]
    D, V, mean = 8_000_000, 140_000, 90.0
    assert abs(D * mean - pm["T"]) <= 0.03 * pm["T"]
    assert abs(V - pm["V"]) <= 0.01 * pm["V"]
    assert mean == pm["T_over_D"]
    assert T3["ClueWeb12"]["V"] == 1_000_000
    small = synth.zipf_corpus(20_000, 140_000, 1.05, 90.0, 0.7, 1)
    assert abs(small.T / small.D - mean) <= 0.03 * mean


def test_zipf_document_prefix_is_the_full_corpus_prefix():
    """The huge-K share is measured on a document prefix drawn without the
    rest of the corpus; it must equal the first documents of the full draw."""
    a = synth.zipf_corpus(3000, 5000, 1.1, 100.0, 1.0, 5)
    b = synth.zipf_corpus(3000, 5000, 1.1, 100.0, 1.0, 5, n_docs=1200)
    p = synth.doc_prefix(a, 1200)
    assert np.array_equal(p.word_ids, b.word_ids) and np.array_equal(p.doc_ids, b.doc_ids)
    assert b.D == 1200
