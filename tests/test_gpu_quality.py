"""The effect of M (Section 6.3) on the NYTimes-shaped corpus at full size,
with the HIP sampler: more MH steps per token reach a higher log likelihood
at the same iteration."""
import numpy as np
import pytest

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


@pytest.mark.timeout(600)
def test_more_mh_steps_converge_faster_at_full_size(W):
    wl = synth.WORKLOADS["nytimes-shape-k1e3"]
    c = wl.make()
    ll = {}
    for M in (1, 2, 4):
        s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, wl.K, M, wl.alpha, wl.beta, seed=1)
        s.init()
        ll[M] = []
        for n in (5, 5, 10):                  # to iterations 5, 10 and 20
            s.iterate(n)
            ll[M].append(s.log_likelihood())
        s.close()
        print(f"M={M}: LL at iterations 5, 10, 20: {np.round(ll[M], 0)}")
    for j in range(3):
        assert ll[1][j] < ll[2][j] < ll[4][j], j
