"""The HIP encoder against the binary64 oracle: gradients, forward output,
input features, proposal weights, and a training run that lowers the loss."""
import numpy as np
import pytest

from oracle import encoder as E
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


def batch(buckets, K, B, seed, vocab=20000):
    rng = np.random.default_rng(seed)
    docs = [rng.integers(0, vocab, int(n)) for n in rng.integers(1, 400, B)]
    theta = rng.dirichlet(np.full(K, 0.2), size=B)
    return docs, theta


def assert_grads_close(names, g_g, g_o, idx=None, rtol=2e-2, atol_frac=2e-3):
    """Element by element: |g - g_o| <= atol + rtol |g_o|, atol a fraction of
    the tensor's largest entry (bf16 operands are rounded at the same points
    on both sides; fp32 against binary64 accumulation can move a rounding by
    one bf16 ulp); the relative Frobenius error is kept as a summary.  For W1
    also the norm of every touched row."""
    for name, gg, go in zip(names, g_g, g_o):
        err = np.linalg.norm(gg - go) / max(np.linalg.norm(go), 1e-30)
        assert err < 5e-3, (name, err)
        atol = atol_frac * float(np.abs(go).max())
        excess = np.abs(gg - go) - (atol + rtol * np.abs(go))
        i = np.unravel_index(int(np.argmax(excess)), go.shape)
        assert excess[i] <= 0, f"{name}: worst entry {i}: gpu {gg[i]!r}, oracle {go[i]!r}, atol {atol:.3g}"
    if idx is not None:
        rows = np.unique(idx)
        rg = np.linalg.norm(g_g[0][rows], axis=1)
        ro = np.linalg.norm(g_o[0][rows], axis=1)
        bad = np.abs(rg - ro) - (1e-2 * ro + 1e-3 * ro.max())
        j = int(np.argmax(bad))
        assert bad[j] <= 0, f"W1 row {rows[j]}: norm gpu {rg[j]!r}, oracle {ro[j]!r}"


def to_dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in arrs]


def test_features_equal_oracle(W):
    rng = np.random.default_rng(1)
    for n in (1, 2, 17, 4000):
        words = rng.integers(0, 100000, n).astype(np.uint32)
        i1, v1 = W.encoder_features(100000, words)
        i2, v2 = E.features(100000, words)
        assert np.array_equal(i1, i2) and np.array_equal(v1, v2)


@pytest.mark.parametrize("buckets,hidden,K,B", [(3000, 200, 70, 37), (5000, 512, 1000, 64)])
def test_gradients_match_oracle(W, buckets, hidden, K, B):
    enc = W.Encoder(buckets, hidden, K, max_batch=B)
    ws = synth.encoder_init_weights(buckets, hidden, K, 3)
    ws[1][:] = 0.05
    ws[3][:] = 0.02
    ws[5][:] = np.linspace(-0.1, 0.1, K, dtype=np.float32)
    enc.set_weights(ws)
    docs, theta = batch(buckets, K, B, 7)
    rowptr, idx, val = E.batch_features(buckets, docs)
    loss_o, q_o, g_o = E.forward_backward(ws, rowptr, idx, val, theta, round=True)
    d_rp, d_idx, d_val, d_th = to_dev(rowptr, idx, val, theta.astype(np.float32))
    loss_g, g_g = enc.gradients(d_rp, d_idx, d_val, d_th)
    assert abs(loss_g - loss_o) <= 1e-4 * abs(loss_o), (loss_g, loss_o)
    q_g = enc.forward(d_rp, d_idx, d_val).cpu().numpy()
    assert np.abs(q_g - q_o).max() <= 1e-4
    assert_grads_close(W.Encoder.NAMES, g_g, g_o, idx)
    # sparse first layer: rows no document touches get no gradient
    untouched = np.setdiff1d(np.arange(buckets), idx)
    assert np.all(g_g[0][untouched] == 0)


def test_gradients_of_a_batch_sliced_from_a_larger_csr(W):
    """Training passes each batch as a slice of the whole corpus's CSR: rowptr
    holds offsets into the full idx and val.  The transpose lists (capacity
    counted from rowptr[0]) must take such a batch, and its forward pass and
    gradients must equal the oracle's on the batch alone."""
    buckets, hidden, K, B = 4000, 256, 90, 24
    enc = W.Encoder(buckets, hidden, K, max_batch=B)
    ws = synth.encoder_init_weights(buckets, hidden, K, 4)
    enc.set_weights(ws)
    docs, theta = batch(buckets, K, 640 + B, 8)
    rowptr, idx, val = E.batch_features(buckets, docs)
    lo = 640                            # a batch deep into the corpus:
    assert rowptr[lo] > 4096 * B        # its offsets alone exceed the lists' capacity
    sub_rp, sub_idx, sub_val = E.batch_features(buckets, docs[lo:lo + B])
    loss_o, q_o, g_o = E.forward_backward(ws, sub_rp, sub_idx, sub_val, theta[lo:lo + B], round=True)
    d_rp, d_idx, d_val, d_th = to_dev(rowptr, idx, val, theta.astype(np.float32))
    loss_g, g_g = enc.gradients(d_rp[lo:lo + B + 1], d_idx, d_val, d_th[lo:lo + B])
    assert abs(loss_g - loss_o) <= 1e-4 * abs(loss_o), (loss_g, loss_o)
    q_g = enc.forward(d_rp[lo:lo + B + 1], d_idx, d_val).cpu().numpy()
    assert np.abs(q_g - q_o).max() <= 1e-4
    assert_grads_close(W.Encoder.NAMES, g_g, g_o, sub_idx)


def test_gradients_past_transpose_capacity(W):
    """The first layer's gradient goes through per-bucket lists that hold 4096
    nonzeros per document of a full batch; a batch with more takes the atomic
    kernel.  One document with ~6000 distinct buckets at max_batch = 1 checks
    that path against the oracle too."""
    buckets, hidden, K = 20000, 128, 40
    enc = W.Encoder(buckets, hidden, K, max_batch=1)
    ws = synth.encoder_init_weights(buckets, hidden, K, 5)
    enc.set_weights(ws)
    rng = np.random.default_rng(9)
    docs = [rng.integers(0, 200000, 9000)]
    theta = rng.dirichlet(np.full(K, 0.2), size=1)
    rowptr, idx, val = E.batch_features(buckets, docs)
    assert rowptr[-1] > 4096
    _, _, g_o = E.forward_backward(ws, rowptr, idx, val, theta, round=True)
    d_rp, d_idx, d_val, d_th = to_dev(rowptr, idx, val, theta.astype(np.float32))
    _, g_g = enc.gradients(d_rp, d_idx, d_val, d_th)
    assert_grads_close(W.Encoder.NAMES, g_g, g_o, idx)


def test_training_lowers_loss(W):
    buckets, hidden, K, B = 4000, 256, 50, 128
    enc = W.Encoder(buckets, hidden, K, max_batch=B, lr=3e-3)
    enc.set_weights(synth.encoder_init_weights(buckets, hidden, K, 5))
    docs, theta = batch(buckets, K, B, 9, vocab=3000)
    rowptr, idx, val = E.batch_features(buckets, docs)
    d = to_dev(rowptr, idx, val, theta.astype(np.float32))
    # soft cross-entropy is bounded below by the entropy of the targets: the
    # KL gap to the targets must shrink
    ent = float(-(theta * np.log(theta)).sum(1).mean())
    first = enc.train_step(*d)
    for _ in range(60):
        last = enc.train_step(*d)
    assert last - ent < 0.5 * (first - ent), (first, last, ent)


def test_proposal_weights(W):
    import torch
    K, B = 1000, 5
    enc = W.Encoder(64, 64, K, max_batch=B)
    rng = np.random.default_rng(2)
    p = rng.dirichlet(np.full(K, 0.1), size=B).astype(np.float32)
    cdf = enc.proposal(torch.from_numpy(p).to("cuda:0"), eps=0.01).cpu().numpy().astype(np.int64)
    e = np.float32(0.01)
    q = ((np.float32(1) - e) * p + e / np.float32(K)).astype(np.float32)
    w = 1 + np.floor(q * np.float32(1 << 20)).astype(np.int64)
    assert np.array_equal(cdf, np.cumsum(w, axis=1))


def test_learned_proposal_gains_over_plain(W):
    """Train the encoder on the sampler's own (document, theta) pairs of an
    LDA-generated corpus, then fold in new documents drawn from the fit: after
    one sweep the learned chain's held-out likelihood beats the plain chain's
    (both chains are exact MH; the learned one starts near the answer)."""
    import torch
    c = synth.lda_corpus(4000, 2000, 16, 120.0, 0.3, 0.02, 77)
    K, M, alpha, beta = 16, 2, 0.3, 0.02
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=1)
    s.init()
    s.iterate(200)
    z, _ = s.assignments()
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, alpha, beta, seed=5)
    buckets, hidden, B = 4096, 128, 200
    counts = np.bincount(c.doc_ids, minlength=c.D)
    docptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
    rowptr, idx, val = W.features_csr(buckets, docptr, c.word_ids[np.argsort(c.doc_ids, kind="stable")])
    d_rp, d_idx, d_val = to_dev(rowptr.astype(np.int32), idx.astype(np.int32), val)
    theta = s.theta(0, c.D)
    enc = W.Encoder(buckets, hidden, K, max_batch=B, lr=3e-3)
    enc.set_weights(synth.encoder_init_weights(buckets, hidden, K, 3, w1_std=1.0))
    for ep in range(25):
        for b0 in range(0, c.D - B + 1, B):
            enc.train_step(d_rp[b0:b0 + B + 1], d_idx, d_val, theta[b0:b0 + B], want_loss=False)
    ev = synth.docs_from_model(c.word_ids, z, c.V, K, alpha, beta, 300, 9, mean_len_log=4.0,
                               sigma=0.5, lo=8, hi=400)
    import bench
    wts = bench.encoder_weights(W, enc, ev[0], ev[1], "cuda:0")
    req = np.arange(300, dtype=np.uint32)
    _, plain1 = gm.foldin(ev[0], ev[1], req, 1, None, 0, ev[2], ev[3])
    _, learn1 = gm.foldin(ev[0], ev[1], req, 1, wts.astype(np.uint32), 2, ev[2], ev[3])
    _, plain50 = gm.foldin(ev[0], ev[1], req, 50, None, 0, ev[2], ev[3])
    gap = plain50.sum() - plain1.sum()
    assert gap > 0
    # the learned chain closes most of the gap to a 50-sweep plain chain in one sweep
    assert learn1.sum() > plain1.sum() + 0.5 * gap, (plain1.sum(), learn1.sum(), plain50.sum())
