"""Pins of the oracle's point estimates (Eq. 4), of its held-out likelihood,
and of the instant-update variant used for the quality study (Section 6.3).

None of these compares the oracle with itself: the estimates are pinned by
normalisation (each theta_d and each phi_k is a distribution over K topics or
V words), by proportionality to counts taken with numpy from the oracle's
assignments, and by limits; the instant-update chain by an exact enumeration
written separately from the paper's definitions, by the collapsed posterior
of Eq. (1) that it must leave invariant, and by a closed form.
"""
import math

import numpy as np
import pytest

import oracle
import synth
import enum_chain
from test_oracle import _chi2_ok


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def trained_oracle(K=5, M=2, alpha=0.3, beta=0.05, iters=3):
    c = synth.random_corpus(3000, 60, 40, seed=21)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=2)
    o.init()
    o.iterate(iters)
    return c, o


# --------------------------------------------------------------------------
# theta_hat and phi_hat (Eq. 4)
# --------------------------------------------------------------------------
def test_theta_rows_are_distributions_proportional_to_counts_plus_alpha():
    c, o = trained_oracle()
    K, alpha = o.K, o.alpha
    th = o.theta()
    z, _ = o.assignments()
    Ld = np.bincount(c.doc_ids, minlength=c.D)
    nonempty = Ld > 0
    # each row sums to one (Eq. 4 normalises over the K topics)
    assert np.allclose(th.sum(1), 1.0, rtol=0, atol=1e-13)
    # and is proportional to C_dk + alpha, counts taken here from z
    cdk = np.zeros((c.D, K))
    np.add.at(cdk, (c.doc_ids, z), 1)
    ratio = th / (cdk + alpha)
    assert np.allclose(ratio, ratio[:, :1], rtol=1e-13, atol=0)
    # sensitivity: the plausible slip L_d + alpha for L_d + K alpha would put
    # the row sums at (L_d + K alpha) / (L_d + alpha), far outside the bound
    slip = (Ld[nonempty] + K * alpha) / (Ld[nonempty] + alpha)
    assert np.abs(slip - 1).min() > 1e-6


def test_phi_columns_are_distributions_over_the_vocabulary():
    c, o = trained_oracle()
    K, beta, V = o.K, o.beta, o.V
    ph = o.phi()
    z, _ = o.assignments()
    # sum over the V declared words of phi_wk is one for every topic
    assert np.allclose(ph.sum(0), 1.0, rtol=0, atol=1e-13)
    cwk = np.zeros((V, K))
    np.add.at(cwk, (c.word_ids, z), 1)
    ratio = ph / (cwk + beta)
    assert np.allclose(ratio, ratio[:1, :], rtol=1e-13, atol=0)


def test_estimates_of_an_empty_document_and_unused_word_are_the_prior():
    c = synth.Corpus(np.array([0, 0, 2], np.uint32), np.array([0, 2, 2], np.uint32), 4, 3)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, 3, 1, 0.4, 0.1, seed=1)
    o.init()
    # document 1 has no tokens: theta = alpha / (K alpha) = 1/K
    assert np.allclose(o.theta(1, 1), 1.0 / 3, rtol=0, atol=1e-15)
    # word 1 never occurs: phi_1k = beta / (C_k + V beta)
    ck = o.topic_counts()
    assert np.allclose(o.phi(1, 1)[0], 0.1 / (ck + 4 * 0.1), rtol=1e-15)


# --------------------------------------------------------------------------
# Held-out likelihood (document completion): p(w | d) = sum_k theta_dk phi_wk
# is a distribution over the V words for every document.
# --------------------------------------------------------------------------
def test_heldout_predictive_distribution_normalises():
    rng = np.random.default_rng(5)
    K, V, T = 4, 9, 80
    w = rng.integers(0, V, T).astype(np.uint32)
    d = rng.integers(0, 6, T).astype(np.uint32)
    z = rng.integers(0, K, T).astype(np.int32)
    z[:20] = 1
    m = oracle.FrozenModel(w, d, z, V, 6, K, 2, 0.35, 0.07)
    # three new documents with chosen assignments (lengths 1, 3, 7)
    zn = np.array([2, 0, 0, 3, 1, 1, 1, 1, 0, 3, 2], np.int32)
    docptr = np.array([0, 1, 4, 11], np.uint64)
    for doc in range(3):
        dp = np.array([0, docptr[doc + 1] - docptr[doc]], np.uint64)
        zd = zn[docptr[doc]:docptr[doc + 1]]
        total = sum(math.exp(m.heldout_ll(dp, zd, np.array([0, 1], np.uint64),
                                          np.array([x], np.uint32))) for x in range(V))
        assert abs(total - 1.0) < 1e-12, (doc, total)
        # sensitivity: theta normalised by L + alpha instead of L + K alpha
        # would give total (L + K alpha) / (L + alpha)
        L = len(zd)
        assert abs((L + K * 0.35) / (L + 0.35) - 1.0) > 1e-3
    # the log of a product is the sum of logs: held-out tokens add up
    ho = np.array([3, 3, 8], np.uint32)
    both = m.heldout_ll(docptr[:2] - docptr[0], zn[:1], np.array([0, 3], np.uint64), ho)
    parts = sum(m.heldout_ll(docptr[:2] - docptr[0], zn[:1], np.array([0, 1], np.uint64), ho[i:i + 1])
                for i in range(3))
    assert abs(both - parts) < 1e-12 * abs(both)


def test_heldout_ll_concentrates_on_the_documents_topic():
    """A long document whose tokens all sit in topic k has theta -> e_k, so the
    held-out likelihood of word x tends to log phi_xk (limit of Eq. 4)."""
    rng = np.random.default_rng(8)
    K, V, T = 3, 5, 60
    w = rng.integers(0, V, T).astype(np.uint32)
    d = rng.integers(0, 4, T).astype(np.uint32)
    z = rng.integers(0, K, T).astype(np.int32)
    beta = 0.2
    m = oracle.FrozenModel(w, d, z, V, 4, K, 1, 0.1, beta)
    cwk = np.zeros((V, K))
    np.add.at(cwk, (w, z), 1)
    ck = np.bincount(z, minlength=K)
    L = 10 ** 7
    for x in range(V):
        got = m.heldout_ll(np.array([0, L], np.uint64), np.full(L, 2, np.int32),
                           np.array([0, 1], np.uint64), np.array([x], np.uint32))
        want = math.log((cwk[x, 2] + beta) / (ck[2] + V * beta))
        assert abs(got - want) < 1e-6, (x, got, want)


# --------------------------------------------------------------------------
# Instant-update variant
# --------------------------------------------------------------------------
INSTANT_CASES = [
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=1, alpha=0.7, beta=0.4, n_iter=1),
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=2, alpha=0.7, beta=0.4, n_iter=2),
    dict(words=[0, 0, 1, 1], docs=[0, 1, 0, 1], V=2, K=2, M=1, alpha=0.3, beta=0.9, n_iter=3),
    dict(words=[0, 1, 2, 1], docs=[0, 0, 0, 1], V=3, K=3, M=1, alpha=0.5, beta=0.2, n_iter=2),
]


@pytest.mark.parametrize("case", INSTANT_CASES)
def test_instant_update_law_matches_enumeration(case):
    w = np.array(case["words"], np.uint32)
    d = np.array(case["docs"], np.uint32)
    K, M, V = case["K"], case["M"], case["V"]
    D = int(d.max()) + 1
    states, pi = enum_chain.instant_distribution_after(list(w), list(d), K, M, case["alpha"],
                                                       case["beta"], V, case["n_iter"])
    index = {s: i for i, s in enumerate(states)}
    n = 12000
    counts = np.zeros(len(states))
    for seed in range(n):
        o = oracle.Oracle(w, d, V, D, K, M, case["alpha"], case["beta"], seed=5000 + seed)
        o.init()
        o.instant_iterate(case["n_iter"])
        z, _ = o.assignments()
        counts[index[tuple(int(x) for x in z)]] += 1
    p = _chi2_ok(counts, pi, n)
    assert p > 1e-4, p


@pytest.mark.parametrize("case", INSTANT_CASES[:2] + INSTANT_CASES[3:])
def test_instant_update_enumeration_leaves_collapsed_posterior_invariant(case):
    """The enumerated instant-update kernel has p(Z | W) of Eq. (1) as a fixed
    point, which the delayed-update kernel does not (reading of Section 4.2)."""
    w, d = case["words"], case["docs"]
    args = (case["K"], case["M"], case["alpha"], case["beta"], case["V"])
    states, P = enum_chain.instant_iteration_matrix(w, d, *args)
    _, post = enum_chain.collapsed_posterior(w, d, case["K"], case["alpha"], case["beta"], case["V"])
    assert np.abs(post @ P - post).max() < 1e-12
    _, Pdel = enum_chain.iteration_matrix(w, d, *args)
    assert np.abs(post @ Pdel - post).max() > 1e-4


def test_instant_update_wright_fisher_case_is_collapsed_gibbs():
    """D = V = 1, alpha = beta: every ratio of Eq. (7) is one, so every step
    accepts and each token is redrawn from its collapsed conditional.  For
    T = K = 2 the stationary P(z1 = z2) is the collapsed posterior's
    (alpha + 1) / (2 alpha + 1) = 2/3 at alpha = 1, where the delayed-update
    chain gives 4/7."""
    n_chains, eq = 6000, 0
    w = np.zeros(2, np.uint32)
    for seed in range(n_chains):
        o = oracle.Oracle(w, w, V=1, D=1, K=2, M=2, alpha=1.0, beta=1.0, seed=seed)
        o.init()
        o.instant_iterate(6)
        assert o.accepted(oracle.PH_DOC) == 2 * 2 * 2
        z, _ = o.assignments()
        eq += int(z[0] == z[1])
    p = 2.0 / 3.0
    se = math.sqrt(p * (1 - p) / n_chains)
    assert abs(eq / n_chains - p) < 4 * se
    assert abs(eq / n_chains - 4.0 / 7.0) > 4 * se


def test_instant_update_keeps_count_invariants():
    c, o = trained_oracle(iters=1)
    o.instant_iterate(2)
    z, _ = o.assignments()
    assert np.array_equal(o.topic_counts(), np.bincount(z, minlength=o.K))
    assert o.iteration == 3
    # the delayed sampler can continue from the instant chain's state
    o.word_phase()
    o.doc_phase()
    z2, _ = o.assignments()
    assert np.array_equal(o.topic_counts(), np.bincount(z2, minlength=o.K))
