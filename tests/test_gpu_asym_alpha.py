"""Parity of the HIP path with the oracle under an asymmetric document-topic
prior alpha_k (Eq. (6)-(7) in their general form): z, the pending proposals,
c_k and the acceptance counts bit for bit after every phase, on corpora whose
documents reach every doc-phase path (16- and 32-lane groups, wave, workgroup,
wide and long rows; dense, packed and two-array count tables; c_k + beta_bar
from LDS or global memory), then the log likelihood within 1e-6 and theta_hat
within 1e-6 relative."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import LL_RTOL, assert_same, mixed_corpus

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def alpha_vector(K, seed, mass=50.0):
    """alpha_k > 0 spread over two orders of magnitude, summing to ~mass."""
    rng = np.random.default_rng(seed)
    a = rng.lognormal(0.0, 1.2, K)
    return (a * (mass / a.sum())).astype(np.float32)


@pytest.mark.parametrize("K,M", [(7, 1), (1000, 2), (1025, 2), (5000, 3), (20000, 4), (70000, 4),
                                 (300000, 2), (64, 4)])
def test_asymmetric_alpha_bit_exact(W, K, M):
    c = mixed_corpus(K + 3 * M)
    a = alpha_vector(K, K + M)
    beta = 0.01
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, 1.0, beta, seed=K + 11 * M)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, 1.0, beta, seed=K + 11 * M)
    s.set_alpha(a)
    o.set_alpha(a)
    s.init()
    o.init()
    assert_same(s, o, "init")
    for it in range(3):
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
    if K <= 16384:
        th = s.theta(0, c.D).cpu().numpy().astype(np.float64)
        th_o = o.theta()
        assert float(np.max(np.abs(th - th_o) / th_o)) <= 1e-6


def test_symmetric_alpha_restored(W):
    """set_alpha(None) returns to the symmetric alpha of the parameters."""
    c = mixed_corpus(5, V=80, D=60, giant_docs=0)
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, 40, 2, 0.3, 0.05, seed=3)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, 40, 2, 0.3, 0.05, seed=3)
    s.set_alpha(alpha_vector(40, 1))
    s.set_alpha(None)
    s.init()
    o.init()
    s.iterate(2)
    o.iterate(2)
    assert_same(s, o, "symmetric again")


def test_set_alpha_errors(W):
    c = mixed_corpus(6, V=50, D=40, giant_docs=0)
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, 8, 2, 0.3, 0.05, seed=3)
    for bad in (np.zeros(8), -np.ones(8), np.full(8, np.nan), np.full(8, np.inf)):
        with pytest.raises(W.WldaError):
            s.set_alpha(bad.astype(np.float32))
    with pytest.raises(ValueError):
        s.set_alpha(np.ones(7, np.float32))
    s.init()
    with pytest.raises(W.WldaError):        # only before the first init
        s.set_alpha(np.ones(8, np.float32))
