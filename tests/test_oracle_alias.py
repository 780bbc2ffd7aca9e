"""The alias-table word proposal of the oracle (Algorithm 2's BuildAlias over
C_w and urn.Draw; alias sampling as Section 2.2 describes it), for the words
with L_w > K.

Pins, none of which reuses the oracle's construction:
* the law of a table, by enumerating every (bin, position) pair of the draw:
  topic k must come out exactly c_k * K times out of K * L;
* three tables worked by hand from the two-pointer sweep;
* the closed form of the sweep's table (running deficits and excesses, the
  construction the GPU uses for K <= 4096) equals the oracle's table;
* the chain law in alias mode against the exact binary64 enumeration (the
  table samples the same law as the inverse CDF, so the chain is unchanged);
* the random-word layout of a draw (bin from the index word, position from
  the same slot on stream 1), rebuilt from Philox and the mixture coin.
"""
import numpy as np
import pytest

import enum_chain
import oracle
from test_oracle import _chi2_ok


def _law_by_enumeration(thr, al, L):
    """Outcome counts of the draw over all K bins and L positions."""
    K = len(thr)
    out = np.zeros(K, np.int64)
    for b in range(K):
        for u in range(L):
            out[b if u < thr[b] else al[b]] += 1
    return out


def _law_by_bins(thr, al, L):
    """The same counts, per bin (bin b gives thr_b to b and L - thr_b to its
    alias); used where K * L is too large to enumerate."""
    K = len(thr)
    out = np.zeros(K, np.int64)
    np.add.at(out, np.arange(K), thr.astype(np.int64))
    np.add.at(out, al.astype(np.int64), L - thr.astype(np.int64))
    return out


def test_hand_worked_tables():
    # c = (3, 1, 0, 0), L = 4, K = 4: weights x = (12, 4, 0, 0) against a mean
    # of 4.  Heavy bin 0 fills light bins 1, 2, 3 (thresholds 4, 0, 0) and is
    # left with 12 - 0 - 4 - 4 = 4 = L, so it keeps itself.
    thr, al = oracle.alias_table([3, 1, 0, 0])
    assert thr.tolist() == [4, 4, 0, 0]
    assert al.tolist() == [0, 0, 0, 0]
    # c = (0, 2, 0, 6), L = 8: x = (0, 8, 0, 24); heavy bin 3 fills bins 0,
    # 1, 2 (thresholds 0, 8, 0), remaining 24 - 8 - 0 - 8 = 8 = L
    thr, al = oracle.alias_table([0, 2, 0, 6])
    assert thr.tolist() == [0, 8, 0, 8]
    assert al.tolist() == [3, 3, 3, 3]
    # two heavy bins: c = (5, 0, 4, 0, 0), L = 9, K = 5: x = (25, 0, 20, 0, 0),
    # mean 9.  Bin 0 (heavy) fills bin 1 (r = 25 - 9 = 16), then bin 3 (r = 7);
    # now r <= 9: bin 0 keeps 7 and gives 2 to the next heavy bin 2 (r = 18),
    # which fills bin 4 (r = 9) and keeps itself.
    thr, al = oracle.alias_table([5, 0, 4, 0, 0])
    assert thr.tolist() == [7, 0, 9, 0, 0]
    assert al.tolist() == [2, 0, 2, 0, 2]


def test_uniform_counts_keep_every_bin():
    thr, al = oracle.alias_table([3] * 7)
    assert thr.tolist() == [21] * 7
    assert al.tolist() == list(range(7))


@pytest.mark.parametrize("seed", range(40))
def test_table_law_is_exact(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 24))
    L = int(rng.integers(K + 1, 4 * K + 40))
    kind = seed % 4
    if kind == 0:       # Dirichlet-multinomial: a few large counts
        c = rng.multinomial(L, rng.dirichlet(np.full(K, 0.3)))
    elif kind == 1:     # one topic holds everything
        c = np.zeros(K, np.int64)
        c[rng.integers(K)] = L
    elif kind == 2:     # near-uniform
        c = rng.multinomial(L, np.full(K, 1.0 / K))
    else:               # many zeros, the rest spread
        p = rng.dirichlet(np.full(K, 1.0)) * (rng.random(K) < 0.3)
        if p.sum() == 0:
            p[0] = 1.0
        c = rng.multinomial(L, p / p.sum())
    thr, al = oracle.alias_table(c)
    assert (thr <= L).all() and (al < K).all()
    assert np.array_equal(_law_by_enumeration(thr, al, L), np.asarray(c) * K)


@pytest.mark.parametrize("K,L", [(1000, 5000), (20000, 60000), (70000, 100000), (1, 9)])
def test_table_law_is_exact_at_kernel_sizes(K, L):
    rng = np.random.default_rng(K)
    c = rng.multinomial(L, rng.dirichlet(np.full(K, 0.05)))
    thr, al = oracle.alias_table(c)
    assert (thr <= L).all() and (al < K).all()
    assert np.array_equal(_law_by_bins(thr, al, L), c * K)


def test_invalid_counts_are_refused():
    with pytest.raises(ValueError):
        oracle.alias_table([0, 0, 0])
    with pytest.raises(ValueError):
        oracle.alias_table([2, -1, 3])


@pytest.mark.parametrize("case", [
    # L_w = K + 1 and larger: word 0 draws from its alias table
    dict(words=[0, 0, 0, 0, 1], docs=[0, 1, 0, 1, 1], V=2, K=3, M=1, alpha=0.5, beta=0.25, n_iter=2),
    dict(words=[0, 0, 0, 1], docs=[0, 1, 0, 1], V=2, K=2, M=1, alpha=0.6, beta=0.3, n_iter=2),
    dict(words=[0, 0, 0, 1, 0], docs=[0, 1, 0, 1, 1], V=2, K=2, M=2, alpha=0.4, beta=0.7, n_iter=2),
])
def test_alias_chain_law_matches_enumeration(case):
    w = np.array(case["words"], np.uint32)
    d = np.array(case["docs"], np.uint32)
    K, M, V = case["K"], case["M"], case["V"]
    D = int(d.max()) + 1
    states, pi = enum_chain.distribution_after(list(w), list(d), K, M, case["alpha"],
                                               case["beta"], V, case["n_iter"])
    index = {s: i for i, s in enumerate(states)}
    n = 12000
    counts = np.zeros(len(states))
    for seed in range(n):
        o = oracle.Oracle(w, d, V, D, K, M, case["alpha"], case["beta"], seed=5000 + seed)
        o.set_word_alias(True)
        o.init()
        o.iterate(case["n_iter"])
        z, _ = o.assignments()
        counts[index[tuple(int(x) for x in z)]] += 1
    p = _chi2_ok(counts, pi, n)
    assert p > 1e-4, p


def _unif24(r):
    return np.float32(np.uint32(r) >> np.uint32(8)) * np.float32(2.0 ** -24)


def _dice(r, n):
    return (int(r) * int(n)) >> 32


def test_draw_word_layout():
    """Proposal i of token t in the word phase: call (i + 1) / 2 of the
    token's counter gives the coin (word 2((i-1) mod 2)) and the index word
    (word 2((i-1) mod 2) + 1); in alias mode the index word picks the bin and
    the same word of stream 1 the position inside it."""
    K, M, alpha, beta, seed = 4, 3, 0.3, 0.01, 77
    rng = np.random.default_rng(3)
    L = 60                                 # one long word (L > K) and a short one
    words = np.r_[np.zeros(L, np.uint32), np.ones(3, np.uint32)]
    docs = rng.integers(0, 5, L + 3).astype(np.uint32)
    o = oracle.Oracle(words, docs, 2, 5, K, M, alpha, beta, seed=seed)
    o.set_word_alias(True)
    o.init()
    o.word_phase()
    z, props = o.csc()                     # column 0 occupies positions 0..L-1
    thr, al = oracle.alias_table(np.bincount(z[:L], minlength=K))
    key = [seed & 0xFFFFFFFF, seed >> 32]
    beta_k = np.float32(K) * np.float32(beta)
    n_count = 0
    for t in range(L):
        for i in range(1, M + 1):
            slot = 2 * ((i - 1) % 2)
            r0 = oracle.philox(key, [t, 1, (1 << 16) | ((i + 1) // 2), 0])
            r1 = oracle.philox(key, [t, 1, (1 << 16) | ((i + 1) // 2), 1])
            coin, iw, uw = r0[slot], r0[slot + 1], r1[slot + 1]
            if _unif24(coin) * (np.float32(L) + beta_k) < np.float32(L):
                b, u = _dice(iw, K), _dice(uw, L)
                want = b if u < thr[b] else al[b]
                n_count += 1
            else:
                want = _dice(iw, K)
            assert props[i - 1, t] == want, (t, i)
    assert n_count > 0.9 * L * M


def test_alias_mode_changes_bits_not_the_counts_it_reads():
    """Alias and inverse-CDF modes draw different proposals for a long word
    from the same state (other random words), and the same ones for short
    words."""
    rng = np.random.default_rng(5)
    K, L = 6, 400
    words = np.r_[np.zeros(L, np.uint32), np.ones(4, np.uint32)]
    docs = rng.integers(0, 9, L + 4).astype(np.uint32)
    outs = []
    for mode in (False, True):
        o = oracle.Oracle(words, docs, 2, 9, K, 2, 0.2, 0.05, seed=11)
        o.set_word_alias(mode)
        o.init()
        o.word_phase()
        outs.append(o.csc())
    (z0, p0), (z1, p1) = outs
    assert np.array_equal(z0, z1)           # same MH outcomes (same doc proposals)
    assert np.array_equal(p0[:, L:], p1[:, L:])
    assert not np.array_equal(p0[:, :L], p1[:, :L])


def _closed_form(c):
    """The sweep's table from running sums alone (the construction the GPU
    uses for K <= 4096): light bins l_1, l_2, ... in topic order with running
    deficit D, heavy bins h_1, h_2, ... with running excess E; light l_k
    aliases the first h_j with E(j) > D(k-1) (none: it keeps itself at L);
    heavy h_j keeps L + E(j) - D(k_j), k_j the first k with D(k) >= E(j),
    and aliases h_{j+1}; the last heavy bin keeps L."""
    c = np.asarray(c, np.int64)
    K, L = len(c), int(c.sum())
    x = c * K
    lights, heavies = np.nonzero(x <= L)[0], np.nonzero(x > L)[0]
    D, E = np.cumsum(L - x[lights]), np.cumsum(x[heavies] - L)
    thr, al = np.zeros(K, np.int64), np.zeros(K, np.int64)
    for r, t in enumerate(lights):
        j = np.searchsorted(E, D[r] - (L - x[t]), side="right")
        thr[t], al[t] = (x[t], heavies[j]) if j < len(heavies) else (L, t)
    for j, t in enumerate(heavies):
        if j == len(heavies) - 1:
            thr[t], al[t] = L, t
        else:
            k = np.searchsorted(D, E[j], side="left")
            thr[t], al[t] = L + E[j] - D[k], heavies[j + 1]
    return thr, al


def test_closed_form_equals_the_sweep():
    rng = np.random.default_rng(11)
    for it in range(600):
        K = int(rng.integers(1, 60))
        L = int(rng.integers(K + 1, 5 * K + 50))
        if it % 3 == 0:
            c = rng.multinomial(L, rng.dirichlet(np.full(K, 0.3)))
        elif it % 3 == 1:
            c = rng.multinomial(L, np.full(K, 1.0 / K))
        else:
            p = rng.dirichlet(np.full(K, 1.0)) * (rng.random(K) < 0.3)
            p[0] += 1e-9
            c = rng.multinomial(L, p / p.sum())
        thr, al = oracle.alias_table(c)
        t2, a2 = _closed_form(c)
        assert np.array_equal(thr, t2) and np.array_equal(al, a2), c
