"""Parity of the HIP path with the CPU oracle (bit-exact assignments).

Every case drives the library through its C ABI (via the ctypes binding) and
the oracle with the same corpus, parameters and seed, then compares z, the
pending proposals, c_k and the acceptance counts element by element after each
phase.  LL must agree within 1e-6 relative (binary64 accumulation in a
different order, device vs host lgamma).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

LL_RTOL = 1e-6


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_08628_amd as W
    W.load_library()
    return W


def make_pair(W, c, K, M, alpha, beta, seed=1):
    s = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=seed)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=seed)
    return s, o


def assert_same(s, o, where=""):
    zs, ps = s.assignments()
    zo, po = o.assignments()
    if not np.array_equal(zs, zo):
        bad = np.nonzero(zs != zo)[0]
        raise AssertionError(f"{where}: z differs at {bad.size} tokens, first {bad[:5]}")
    if not np.array_equal(ps, po):
        bad = np.nonzero((ps != po).any(0))[0]
        raise AssertionError(f"{where}: proposals differ at {bad.size} tokens, first {bad[:5]}")
    assert np.array_equal(s.topic_counts(), o.topic_counts()), where


def mixed_corpus(seed, V=300, D=220, s=1.2, giant_docs=2):
    """Zipf words (a few columns longer than one workgroup's share), lognormal
    documents plus a few giant ones, some empty documents and unused words."""
    rng = np.random.default_rng(seed)
    lens = np.maximum(1, rng.lognormal(np.log(250) - 0.5, 1.0, D).astype(int))
    lens[:giant_docs] = 6000           # longer than one workgroup (doc long path)
    lens[giant_docs:giant_docs + 5] = 1500   # workgroup path
    lens[-3:] = 0                      # empty documents
    T = int(lens.sum())
    w = np.arange(1, V + 1, dtype=float) ** -s
    w[-7:] = 0                         # words that never occur
    w /= w.sum()
    words = rng.choice(V, size=T, p=w).astype(np.uint32)
    docs = np.repeat(np.arange(D, dtype=np.uint32), lens)
    perm = rng.permutation(T)          # input order is arbitrary
    return synth.Corpus(words[perm], docs[perm], V, D)


def test_tiny_lda_corpus_50_iterations(W):
    wl = synth.WORKLOADS["tiny-lda-k16"]
    c = wl.make()
    s, o = make_pair(W, c, wl.K, wl.M, wl.alpha, wl.beta, seed=1)
    s.init()
    o.init()
    assert_same(s, o, "init")
    s.word_phase()
    o.word_phase()
    assert_same(s, o, "word phase 1")
    assert s.accepted(1) == o.accepted(1)
    s.doc_phase()
    o.doc_phase()
    assert_same(s, o, "doc phase 1")
    assert s.accepted(2) == o.accepted(2)
    for it in (10, 50):
        n = it - o.iteration
        s.iterate(n)
        o.iterate(n)
        assert_same(s, o, f"iteration {it}")
        assert s.iteration == o.iteration == it
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= LL_RTOL * abs(ll_o), (ll_s, ll_o)


# record formats: 32-bit with 16-bit fields (M=1, K<=65536), 10-bit (M=2,
# K<=1024), 8-bit (M=3, K<=256), 6-bit (M=4, K<=64); else, for K <= 65536,
# 16-bit fields in two (M=2, 3) or three (M=4) 32-bit words; else 21-bit
# fields in one (M <= 2) or two 64-bit words
@pytest.mark.parametrize("K,M", [(7, 1), (65536, 1), (1000, 2), (1024, 2), (1025, 2), (256, 3),
                                 (5000, 3), (64, 4), (20000, 4), (300000, 2), (1000000, 2), (2000, 4),
                                 (100000, 3), (70000, 4), (65536, 4)])
def test_all_paths_bit_exact(W, K, M):
    c = mixed_corpus(K + M)
    alpha, beta = 50.0 / K, 0.01
    s, o = make_pair(W, c, K, M, alpha, beta, seed=K * 7 + M)
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


@pytest.mark.parametrize("case", ["one_token", "one_doc_one_word", "k1", "all_same_cell",
                                  "empty_rows_cols", "ragged_tail", "ragged_tail_m4"])
def test_edge_cases(W, case):
    rng = np.random.default_rng(3)
    if case == "one_token":
        c = synth.Corpus(np.array([4], np.uint32), np.array([2], np.uint32), 5, 3)
        K, M = 3, 2
    elif case == "one_doc_one_word":
        c = synth.Corpus(np.zeros(777, np.uint32), np.zeros(777, np.uint32), 1, 1)
        K, M = 5, 2
    elif case == "k1":
        c = synth.random_corpus(5000, 40, 30, seed=5)
        K, M = 1, 2
    elif case == "all_same_cell":      # one column and one row, both long
        c = synth.Corpus(np.full(12000, 3, np.uint32), np.full(12000, 1, np.uint32), 4, 2)
        K, M = 50, 2
    elif case == "empty_rows_cols":
        w = rng.integers(0, 10, 3000).astype(np.uint32) * 10      # 90% of words unused
        d = rng.integers(0, 20, 3000).astype(np.uint32) * 5       # 80% of docs empty
        c = synth.Corpus(w, d, 100, 100)
        K, M = 64, 2
    else:                              # lengths straddling every bin boundary
        # 16-lane groups 128, 32-lane groups 256, wave 512; block 2048 (1024
        # for M > 2); wide 4096 (2048); long path
        lens = [511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097,
                1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257]
        d = np.repeat(np.arange(len(lens), dtype=np.uint32), lens)
        w = np.concatenate([np.full(L, i, np.uint32) for i, L in enumerate(lens)])
        w = w[rng.permutation(len(w))]
        c = synth.Corpus(w, d, len(lens), len(lens))
        K, M = (200, 2) if case == "ragged_tail" else (200, 4)
    s, o = make_pair(W, c, K, M, 0.3, 0.02, seed=11)
    s.init()
    o.init()
    assert_same(s, o, "init")
    for it in range(2):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, f"{case} word {it}")
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, f"{case} doc {it}")
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= LL_RTOL * abs(ll_o) + 1e-9, (ll_s, ll_o)


def test_wright_fisher_case_accepts_everything(W):
    """D = V = 1, alpha = beta: both Eq. (7) ratios are exactly 1."""
    c = synth.Corpus(np.zeros(3000, np.uint32), np.zeros(3000, np.uint32), 1, 1)
    s = W.Sampler(c.word_ids, c.doc_ids, 1, 1, 4, 2, 1.0, 1.0, seed=3)
    s.init()
    for _ in range(3):
        s.word_phase()
        assert s.accepted(1) == 2 * 3000
        s.doc_phase()
        assert s.accepted(2) == 2 * 3000


def test_checkpoint_resume_and_order_errors(W):
    c = mixed_corpus(9, V=120, D=90, giant_docs=1)
    K, M = 100, 2
    a = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, 0.5, 0.01, seed=4)
    with pytest.raises(W.WldaError) as e:
        a.word_phase()
    assert e.value.code == -4
    a.init()
    with pytest.raises(W.WldaError):
        a.doc_phase()
    a.iterate(2)
    a.word_phase()
    blob = a.save_state()
    a.doc_phase()
    a.iterate(2)
    b = W.Sampler(c.word_ids, c.doc_ids, c.V, c.D, K, M, 0.5, 0.01, seed=4)
    b.load_state(blob)
    b.doc_phase()
    b.iterate(2)
    za, pa = a.assignments()
    zb, pb = b.assignments()
    assert np.array_equal(za, zb) and np.array_equal(pa, pb)
    assert a.iteration == b.iteration == 5


def test_set_assignments_matches_oracle(W):
    c = mixed_corpus(9, V=120, D=90, giant_docs=1)
    K, M = 100, 2
    s, o = make_pair(W, c, K, M, 0.5, 0.01, seed=4)
    s.init()
    o.init()
    zo, po = o.assignments()
    rng = np.random.default_rng(0)
    z2 = ((zo + rng.integers(0, 3, zo.shape)) % K).astype(np.int32)
    p2 = ((po + 1) % K).astype(np.int32)
    s.set_assignments(z2, p2)
    _, _, _, inv = o.layout()
    zc = np.empty_like(z2)
    zc[inv] = z2
    pc = np.empty_like(p2)
    pc[:, inv] = p2
    o.set_csc_state(zc, pc)
    assert_same(s, o, "after set")
    for _ in range(2):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, "word after set")
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, "doc after set")


@pytest.mark.parametrize("block_kib,first_bin", [("0", "0"), ("16", "0"), ("4096", "0"), ("1024", "2"),
                                                ("1024", "1")])
@pytest.mark.parametrize("K,M", [(1000, 2), (50, 4)])
def test_record_layouts_bit_exact(W, block_kib, first_bin, K, M, monkeypatch):
    """The record layout (plain CSC order, or blocked by documents with tiny
    or large blocks) and the launch shape (segments of every length in
    wavefront-wide or wider groups only) change where records live and who
    processes them, never the chain."""
    monkeypatch.setenv("WLDA_DOC_BLOCK_KIB", block_kib)
    monkeypatch.setenv("WLDA_FIRST_BIN", first_bin)
    c = mixed_corpus(K + M + 3)
    s, o = make_pair(W, c, K, M, 50.0 / K, 0.01, seed=5)
    s.init()
    o.init()
    assert_same(s, o, "init")
    for it in range(2):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, f"word phase {it + 1}")
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, f"doc phase {it + 1}")
    ll_s, ll_o = s.log_likelihood(), o.log_likelihood()
    assert abs(ll_s - ll_o) <= LL_RTOL * abs(ll_o), (ll_s, ll_o)


def head_word_corpus(seed, head_len, V=300, D=220):
    """mixed_corpus plus one word of head_len tokens spread over the
    documents: a column far longer than one workgroup's share."""
    c = mixed_corpus(seed, V, D)
    rng = np.random.default_rng(seed + 1)
    head = V - 8                       # a word of the Zipf tail
    docs = rng.integers(0, D - 3, head_len).astype(np.uint32)
    words = np.concatenate([c.word_ids, np.full(head_len, head, np.uint32)])
    docs = np.concatenate([c.doc_ids, docs])
    perm = rng.permutation(len(words))
    return synth.Corpus(words[perm], docs[perm], V, D)


@pytest.mark.parametrize("K,M,head", [(20000, 2, 60000), (40000, 4, 100000), (20000, 1, 70000),
                                      (300000, 2, 400000)])
def test_long_column_longer_than_large_K(W, K, M, head):
    """A column longer than K with K above the LDS limits of the long path
    (16384): its word proposals take the inverse CDF through prefix counts in
    global memory, and its updated counts are added with global atomics."""
    c = head_word_corpus(K + M, head)
    assert np.bincount(c.word_ids, minlength=c.V).max() > K
    s, o = make_pair(W, c, K, M, 50.0 / K, 0.01, seed=K + 3 * M)
    s.init()
    o.init()
    assert_same(s, o, "init")
    for it in range(2):
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


# K around the lengths of each bin: 16-lane groups (<= 128 tokens), 32-lane
# groups (256), wave (512), block (2048, or 1024 for M > 2), wide (4096 or
# 2048) and the long path; columns of K - 1, K
# and K + 1 tokens straddle the switch from random positioning to the
# inverse CDF
@pytest.mark.parametrize("K,M", [(60, 2), (200, 2), (400, 2), (1500, 2), (3000, 2), (6000, 2),
                                 (100, 4), (300, 4), (800, 4), (1800, 4), (3000, 4)])
def test_word_cdf_boundary_in_every_bin(W, K, M):
    rng = np.random.default_rng(K + M)
    D = 60
    lens = [K - 1, K, K + 1]
    words = [np.full(L, i, np.uint32) for i, L in enumerate(lens)]
    words.append(rng.integers(3, 40, 4000).astype(np.uint32))     # background words
    w = np.concatenate(words)
    d = rng.integers(0, D, len(w)).astype(np.uint32)
    c = synth.Corpus(w, d, 40, D)
    s, o = make_pair(W, c, K, M, 0.5, 0.05, seed=17)
    s.init()
    o.init()
    for it in range(2):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, f"word phase {it + 1}")
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, f"doc phase {it + 1}")


@pytest.mark.parametrize("M", [2, 4])
def test_topic_histogram_counter_overflow(W, M, monkeypatch):
    """Above 4096 topics the row kernels count c_k of the new Z in 16-bit LDS
    counters that move 0x8000 to the global count each time they reach it.
    With every token on one topic and eight workgroups per bin, each
    workgroup adds that topic 2^16 times or more, so the carry runs several
    times; z, proposals and c_k must still match the oracle exactly."""
    monkeypatch.setenv("WLDA_SEG_BLOCKS", "768,768,768,1024,768,8,8,8,8,8")
    K = 5000
    rng = np.random.default_rng(40 + M)
    D = 12000
    hi = 64 if M > 2 else 128          # every row in the 16-lane groups
    lens = rng.integers(20, hi + 1, D)
    T = int(lens.sum())
    docs = np.repeat(np.arange(D, dtype=np.uint32), lens)
    words = rng.integers(0, 50, T).astype(np.uint32)
    perm = rng.permutation(T)
    c = synth.Corpus(words[perm], docs[perm], 50, D)
    s, o = make_pair(W, c, K, M, 0.01, 0.01, seed=6)
    s.init()
    o.init()
    z0 = np.zeros(T, np.int32)
    p0 = np.zeros((M, T), np.int32)
    s.set_assignments(z0, p0)
    o.set_csc_state(z0, p0)             # all equal: input and CSC order agree
    for it in range(2):
        s.word_phase()
        o.word_phase()
        assert_same(s, o, f"word phase {it + 1}")
        s.doc_phase()
        o.doc_phase()
        assert_same(s, o, f"doc phase {it + 1}")
        if it == 0:     # about 1.5 carries per workgroup in the first doc phase at least
            assert o.topic_counts()[0] >= 8 * 0x8000 * 1.5
