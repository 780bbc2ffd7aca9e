"""The continuous-batching server: every result equals the oracle's fold-in of
that document alone (bit-exact z, held-out LL to 1e-9), whatever else was in
flight; admission respects the slot and pool limits."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_foldin import trained, synthetic_weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def requests(V, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        L = int(np.clip(rng.lognormal(np.log(150), 0.9), 1, 2500))
        out.append((1000 + 3 * r, rng.integers(0, V, L).astype(np.uint32),
                    rng.integers(0, V, int(rng.integers(0, 30))).astype(np.uint32)))
    return out


def test_server_matches_oracle_under_admission_pressure(W):
    K, M, S = 50, 2, 3
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    om = oracle.FrozenModel(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    reqs = requests(c.V, 80, 3)
    wts = synthetic_weights(80, K, 6)
    # small pool and few slots: requests wait, are admitted as others retire
    srv = W.Server(gm, None, max_docs=12, pool_tokens=4000, pool_heldout=400, sweeps=S,
                   learned_steps=2)
    learned = {}
    sub = 0
    results = {}
    steps = 0
    while len(results) < len(reqs):
        if sub < len(reqs):                 # a few arrivals per step
            for _ in range(3):
                if sub == len(reqs):
                    break
                rid, words, ho = reqs[sub]
                use = sub % 2 == 1
                learned[rid] = wts[sub] if use else None
                srv.submit(rid, words, ho, weights=learned[rid])
                sub += 1
        active, pending = srv.step()
        assert active <= 12
        for r in srv.poll():
            results[r["req_id"]] = r
        steps += 1
        assert steps < 10000
    for rid, words, ho in reqs:
        r = results[rid]
        assert r["n_tokens"] == len(words) and r["sweeps"] == S
        assert r["learned"] == (learned[rid] is not None)
        zs = srv.take_z(rid, len(words))
        zo, _ = om.foldin(np.array([0, len(words)], np.uint64), words, [rid], S,
                          None if learned[rid] is None else learned[rid][None, :],
                          2 if learned[rid] is not None else 0)
        assert np.array_equal(zs, zo), rid
        ho_ll = om.heldout_ll(np.array([0, len(words)], np.uint64), zo,
                              np.array([0, len(ho)], np.uint64), ho)
        assert abs(r["heldout_ll"] - ho_ll) <= 1e-9 * max(1.0, abs(ho_ll))
        assert r["arrival_s"] <= r["admit_s"] <= r["done_s"]


def test_server_with_encoder_alone_equals_in_mix(W):
    import torch
    K, M, S = 50, 2, 2
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    enc = W.Encoder(2000, 128, K, max_batch=16)
    enc.set_weights(synth.encoder_init_weights(2000, 128, K, 2))
    reqs = requests(c.V, 30, 8)
    mixed = W.Server(gm, enc, max_docs=16, pool_tokens=20000, pool_heldout=1000, sweeps=S)
    for rid, words, ho in reqs:
        mixed.submit(rid, words, ho)
    got = {}
    while len(got) < len(reqs):
        mixed.step()
        for r in mixed.poll():
            got[r["req_id"]] = mixed.take_z(r["req_id"], r["n_tokens"])
            assert r["learned"]
    for rid, words, ho in reqs[::7]:
        alone = W.Server(gm, enc, max_docs=1, pool_tokens=5000, pool_heldout=100, sweeps=S)
        alone.submit(rid, words, ho)
        res = []
        while not res:
            alone.step()
            res = alone.poll()
        assert np.array_equal(alone.take_z(rid, len(words)), got[rid])


def test_server_encode_ahead_with_requests_waiting_several_steps(W):
    """Few slots, a larger encoder batch and many sweeps: requests are encoded
    ahead into a stage and wait there for several steps while the stages are
    reused; each result still equals the request's result alone."""
    K, M, S = 50, 2, 5
    c, z = trained(K, M)
    gm = W.Model(c.word_ids, c.doc_ids, z, c.V, c.D, K, M, 50.0 / K, 0.01, seed=7)
    enc = W.Encoder(2000, 128, K, max_batch=16)
    enc.set_weights(synth.encoder_init_weights(2000, 128, K, 4))
    reqs = requests(c.V, 40, 12)
    mixed = W.Server(gm, enc, max_docs=4, pool_tokens=20000, pool_heldout=1000, sweeps=S)
    for rid, words, ho in reqs:
        mixed.submit(rid, words, ho)
    got, steps = {}, 0
    while len(got) < len(reqs):
        active, pending = mixed.step()
        assert active <= 4
        steps += 1
        assert steps < 1000
        for r in mixed.poll():
            got[r["req_id"]] = mixed.take_z(r["req_id"], r["n_tokens"])
    assert steps >= (len(reqs) // 4) * (S + 1)
    for rid, words, ho in reqs[1::6]:
        alone = W.Server(gm, enc, max_docs=1, pool_tokens=5000, pool_heldout=100, sweeps=S)
        alone.submit(rid, words, ho)
        res = []
        while not res:
            alone.step()
            res = alone.poll()
        assert np.array_equal(alone.take_z(rid, len(words)), got[rid]), rid
