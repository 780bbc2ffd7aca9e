"""The allocation-free fold-in entry point (wlda_foldin_batch_static) against
the workspace entry point (wlda_foldin_batch) through the C ABI: identical
assignments and held-out likelihoods on two calls in a row, the second with a
smaller batch (the static device array keeps the first call's contents), in
plain and learned mode; a batch beyond the array's size is refused."""
import numpy as np
import pytest

import synth
from test_gpu_foldin import trained, new_docs, synthetic_weights

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20     # WLDA_FOLDIN_STATIC_BYTES in include/warplda.h


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


@pytest.mark.parametrize("learned", [False, True])
def test_static_foldin_equals_workspace_foldin(W, learned):
    K, M = 50, 2
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    for call, (n, seed) in enumerate([(60, 21), (9, 22)]):     # second call smaller
        docptr, words = new_docs(c.V, n, seed)
        rng = np.random.default_rng(seed)
        ho_len = rng.integers(0, 40, n)
        hoptr = np.concatenate([[0], np.cumsum(ho_len)]).astype(np.uint64)
        how = rng.integers(0, c.V, int(hoptr[-1])).astype(np.uint32)
        req = np.arange(100 * call, 100 * call + n, dtype=np.uint32)
        wts = synthetic_weights(n, K, seed) if learned else None
        ls = 2 if learned else 0
        z_ws, ho_ws = gm.foldin(docptr, words, req, 4, wts, ls, hoptr, how)
        z_st, ho_st = gm.foldin_static(docptr, words, req, 4, wts, ls, hoptr, how)
        assert np.array_equal(z_ws, z_st), call
        assert np.array_equal(ho_ws, ho_st), call
    gm.close()


def test_static_foldin_rejects_a_batch_beyond_its_array(W):
    K, M = 50, 2
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    # (2 + 2M) * 4 bytes per token: 3M tokens need 72 MB > 64 MiB
    n, L = 1500, 2000
    docptr = (np.arange(n + 1) * L).astype(np.uint64)
    words = np.zeros(n * L, np.uint32)
    with pytest.raises(W.WldaError) as e:
        gm.foldin_static(docptr, words, np.arange(n, dtype=np.uint32), 1)
    assert e.value.code == -2
    # and works again afterwards
    docptr, words = new_docs(c.V, 5, 3)
    req = np.arange(5, dtype=np.uint32)
    assert np.array_equal(gm.foldin(docptr, words, req, 2)[0], gm.foldin_static(docptr, words, req, 2)[0])
    gm.close()
