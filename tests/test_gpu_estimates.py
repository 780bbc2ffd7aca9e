"""theta_hat and phi_hat of Eq. (4) from the HIP library against the oracle's
binary64 values on the same sampler state.  The library rounds numerator and
denominator to binary32 once each and divides, so each entry lies within a
few binary32 ulps (relative 1e-6) of the exact value."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import make_pair, mixed_corpus, assert_same

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def worst(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


@pytest.mark.parametrize("K,M", [(1000, 2), (50, 4), (9000, 1)])
def test_theta_and_phi_match_oracle(W, K, M):
    c = mixed_corpus(K + 5 * M)
    s, o = make_pair(W, c, K, M, 50.0 / K, 0.01, seed=9)
    s.init()
    o.init()
    s.iterate(2)
    o.iterate(2)
    assert_same(s, o, "state")
    th = s.theta(0, c.D).cpu().numpy().astype(np.float64)
    ph = s.phi(0, c.V).cpu().numpy().astype(np.float64)
    th_o, ph_o = o.theta(), o.phi()
    assert worst(th, th_o) <= RTOL, worst(th, th_o)
    assert worst(ph, ph_o) <= RTOL, worst(ph, ph_o)
    # sub-ranges (documents and words past the first)
    assert np.array_equal(s.theta(7, 30).cpu().numpy(), th[7:37].astype(np.float32))
    assert np.array_equal(s.phi(11, 50).cpu().numpy(), ph[11:61].astype(np.float32))


def test_estimates_reject_bad_ranges(W):
    c = mixed_corpus(3, V=50, D=40, giant_docs=0)
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, 20, 2, 0.5, 0.01, seed=1)
    with pytest.raises(W.WldaError) as e:
        s.phi(0, 10)
    assert e.value.code == -4          # before init
    s.init()
    with pytest.raises(W.WldaError) as e:
        s.phi(45, 10)
    assert e.value.code == -1
    with pytest.raises(W.WldaError) as e:
        s.theta(35, 10)
    assert e.value.code == -1
