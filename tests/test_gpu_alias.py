"""Parity of the alias-table word proposal (WLDA_WORD_ALIAS: Walker's alias
table over the updated c_w for words with L_w > K, Algorithm 2's BuildAlias
and urn.Draw) with the oracle in the same mode: z, the pending proposals, c_k
and the acceptance counts bit for bit after every phase."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import LL_RTOL, assert_same, head_word_corpus, mixed_corpus

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def run_pair(W, c, K, M, seed, iters=3):
    alpha, beta = 50.0 / K, 0.01
    print(f"alias parity K={K} M={M} T={len(c.word_ids)} seed={seed}", flush=True)
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=seed, word_alias=True)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=seed)
    o.set_word_alias(True)
    s.init()
    o.init()
    assert_same(s, o, "init")
    for it in range(iters):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, f"word phase {it + 1}")
        assert s.accepted(1) == o.accepted(1)
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, f"doc phase {it + 1}")
        assert s.accepted(2) == o.accepted(2)
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= LL_RTOL * abs(ll_o), (ll_s, ll_o)
    return s


# small K (most words longer than K: hundreds of long words, also ones of
# K + 1 tokens), the record formats of M = 1..4 (tables built by a whole
# workgroup in closed form, K <= 4096); below, K = 6000 (one lane sweeps in
# LDS), K past the LDS limits of the long path and K > 65535 (one thread per
# word sweeps in global memory; 32-bit compact topics, 21-bit fields)
@pytest.mark.parametrize("K,M", [(8, 2), (1, 1), (60, 1), (1000, 2), (256, 3), (2000, 4)])
def test_alias_word_proposals_bit_exact(W, K, M):
    c = mixed_corpus(K + 17 * M)
    assert np.bincount(c.word_ids, minlength=c.V).max() > K
    run_pair(W, c, K, M, seed=K * 5 + M)


@pytest.mark.parametrize("K,M,head", [(20000, 2, 60000), (70000, 3, 100000), (4096, 2, 30000),
                                      (6000, 4, 40000)])
def test_alias_long_column_longer_than_large_K(W, K, M, head):
    c = head_word_corpus(K + M, head)
    run_pair(W, c, K, M, seed=K + M, iters=2)


def test_alias_flag_changes_the_draws(W):
    """Same corpus and seed with and without the flag: the word proposals of
    words with L_w > K differ (other random words), the assignments after the
    first word phase do not (the MH pass reads the same doc proposals)."""
    c = mixed_corpus(99)
    K, M = 100, 2
    outs = []
    for alias in (False, True):
        s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, 0.5, 0.01, seed=4, word_alias=alias)
        s.init()
        s.word_phase()
        outs.append(s.assignments())
    (z0, p0), (z1, p1) = outs
    assert np.array_equal(z0, z1)
    assert not np.array_equal(p0, p1)
