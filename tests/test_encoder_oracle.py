"""Pins of the encoder oracle: exact (unrounded) gradients against central
finite differences, the bfloat16 rounding rule, and the input features."""
import numpy as np

from oracle import encoder as E
import synth


def test_bf16_rounding_rule():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -7 + 2 ** -9, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0 + 2 ** -7, 0.0])
    assert np.array_equal(E.bf16(x), want)


def test_features_definition():
    idx, val = E.features(1000, [5, 7, 5, 5])
    b = lambda w: ((w * 0x9E3779B1) % 2 ** 32 * 1000) >> 32
    want = {}
    for w in (5, 7, 5, 5):
        want[b(w)] = want.get(b(w), 0) + 1
    assert list(idx) == sorted(want)
    for i, v in zip(idx, val):
        assert v == np.float32(want[int(i)]) / np.float32(4)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    buckets, hidden, K, B = 40, 6, 5, 3
    ws = [w.astype(np.float64) for w in synth.encoder_init_weights(buckets, hidden, K, 1)]
    ws[1] += 0.1
    ws[3] += 0.05
    docs = [rng.integers(0, 500, n) for n in (7, 3, 11)]
    rowptr, idx, val = E.batch_features(buckets, docs)
    theta = rng.dirichlet(np.ones(K), size=B)
    loss, _, grads = E.forward_backward(ws, rowptr, idx, val, theta, round=False)
    h = 1e-6
    for p_i, g in enumerate(grads):
        flat = ws[p_i].reshape(-1)
        gflat = g.reshape(-1)
        # every entry of small tensors, a sample of W1 (rows the batch touches)
        cand = np.arange(flat.size)
        if p_i == 0:
            rows = np.unique(idx)
            cand = (rows[:, None] * hidden + np.arange(hidden)).reshape(-1)
        for j in cand:
            old = flat[j]
            flat[j] = old + h
            lp, _, _ = E.forward_backward(ws, rowptr, idx, val, theta, round=False)
            flat[j] = old - h
            lm, _, _ = E.forward_backward(ws, rowptr, idx, val, theta, round=False)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[j]) <= 1e-6 + 1e-5 * abs(fd), (p_i, j, fd, gflat[j])
    # untouched W1 rows get exactly zero gradient
    untouched = np.setdiff1d(np.arange(buckets), idx)
    assert np.all(grads[0][untouched] == 0)


def test_rounded_path_is_the_exact_path_up_to_bf16_rounding():
    """The rounded mode (operands of every product rounded to bfloat16 where
    the GPU rounds them) uses the same formulas as the exact mode that the
    finite differences pin: its loss and probabilities agree to bfloat16
    precision, and every gradient points the same way (cosine > 0.95; the
    output error p - theta is small and rounds coarsely, so the backward
    products differ by up to ~20%).  A dropped term, a wrong sign or a
    transposed operand in the rounded path would show."""
    rng = np.random.default_rng(3)
    buckets, hidden, K, B = 300, 64, 20, 16
    ws = [w.astype(np.float64) for w in synth.encoder_init_weights(buckets, hidden, K, 2)]
    ws[1] += 0.05
    ws[3] += 0.02
    ws[5] += np.linspace(-0.2, 0.2, K)
    docs = [rng.integers(0, 5000, n) for n in rng.integers(5, 200, B)]
    rowptr, idx, val = E.batch_features(buckets, docs)
    theta = rng.dirichlet(np.full(K, 0.3), size=B)
    l_r, q_r, g_r = E.forward_backward(ws, rowptr, idx, val, theta, round=True)
    l_e, q_e, g_e = E.forward_backward(ws, rowptr, idx, val, theta, round=False)
    assert abs(l_r - l_e) <= 2e-2 * abs(l_e)
    assert np.abs(q_r - q_e).max() <= 2e-2
    for gr, ge in zip(g_r, g_e):
        cos = float(np.sum(gr * ge) / (np.linalg.norm(gr) * np.linalg.norm(ge)))
        err = np.linalg.norm(gr - ge) / np.linalg.norm(ge)
        assert cos > 0.95 and err < 0.3, (cos, err)
    # and they are not the same computation: rounding is applied
    assert any(not np.array_equal(gr, ge) for gr, ge in zip(g_r, g_e))
