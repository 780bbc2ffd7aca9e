"""Pins of the oracle's asymmetric document-topic prior alpha_k (the general
form of Eq. (6)-(7)): doc proposals q_doc(k) ~ C_dk + alpha_k, the word
proposal's acceptance rate with alpha_c and alpha_s, the log likelihood and
theta_hat with alpha_k.  None of these compares the oracle with itself: the
chain's law against exact enumeration, the frozen-count kernels against
Eq. (5), the log likelihood against normalisation, theta_hat against its
definition."""
import itertools
import math

import numpy as np
import pytest

import enum_chain
import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _chi2_p(counts, probs, n, min_expected=5.0):
    from scipy import stats
    mask = probs * n >= min_expected
    obs = np.append(counts[mask], counts[~mask].sum())
    exp = np.append(probs[mask] * n, probs[~mask].sum() * n)
    if exp[-1] < 1e-9:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chi2.sf(((obs - exp) ** 2 / exp).sum(), len(obs) - 1)


CASES = [
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=1, alpha=[0.2, 1.6, 0.7], beta=0.4, n_iter=1),
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=2, alpha=[1.1, 0.15, 0.5], beta=0.3, n_iter=2),
    # a column longer than K (inverse-CDF word proposals) and a long row
    dict(words=[0, 0, 0, 1], docs=[0, 0, 0, 1], V=2, K=2, M=1, alpha=[0.25, 2.0], beta=0.5, n_iter=2),
]


@pytest.mark.parametrize("case", CASES)
def test_asymmetric_chain_law_matches_enumeration(case):
    w = np.array(case["words"], np.uint32)
    d = np.array(case["docs"], np.uint32)
    K, M, V = case["K"], case["M"], case["V"]
    a = np.array(case["alpha"], np.float32)
    states, pi = enum_chain.distribution_after(list(w), list(d), K, M, a.astype(np.float64),
                                               case["beta"], V, case["n_iter"])
    index = {s: i for i, s in enumerate(states)}
    n = 12000
    counts = np.zeros(len(states))
    for seed in range(n):
        o = oracle.Oracle(w, d, V, int(d.max()) + 1, K, M, 1.0, case["beta"], seed=5000 + seed)
        o.set_alpha(a)
        o.init()
        o.iterate(case["n_iter"])
        z, _ = o.assignments()
        counts[index[tuple(int(x) for x in z)]] += 1
    assert _chi2_p(counts, pi, n) > 1e-4


def test_enumeration_tells_asymmetric_from_symmetric_alpha():
    """The pin above can fail: replacing alpha_k by their mean moves the law
    by far more than the test's resolution."""
    c = CASES[0]
    a = np.array(c["alpha"])
    _, right = enum_chain.distribution_after(c["words"], c["docs"], c["K"], c["M"], a, c["beta"],
                                             c["V"], 2)
    _, wrong = enum_chain.distribution_after(c["words"], c["docs"], c["K"], c["M"], a.mean(),
                                             c["beta"], c["V"], 2)
    assert 0.5 * np.abs(right - wrong).sum() > 4 * np.sqrt(len(right) / 12000)


def test_frozen_count_chain_targets_eq5_with_alpha_k():
    """With Z held fixed, the doc-proposal kernel (prior part drawn from
    alpha_k / alpha_bar), the word-proposal kernel (rate with alpha_c,
    alpha_s) and both together leave q(k) ~ (C_dk + alpha_k)(C_wk + beta) /
    (C_k + V beta) invariant."""
    rng = np.random.default_rng(9)
    T = 24
    w = rng.integers(0, 4, T).astype(np.uint32)
    d = rng.integers(0, 3, T).astype(np.uint32)
    K, beta, V = 4, 0.3, 4
    a = np.array([0.1, 2.5, 0.6, 1.2], np.float32)
    o = oracle.Oracle(w, d, V, 3, K, 2, 1.0, beta, seed=78)
    o.set_alpha(a)
    zin = rng.integers(0, K, T).astype(np.int32)
    zin[:8] = 0
    o.init()
    _, _, _, inv = o.layout()
    zcsc = np.empty(T, np.int32)
    zcsc[inv] = zin
    o.set_csc_state(zcsc)
    ck = np.bincount(zin, minlength=K).astype(float)
    for t_in in [0, 11, 23]:
        cd = np.bincount(zin[d == d[t_in]], minlength=K).astype(float)
        cw = np.bincount(zin[w == w[t_in]], minlength=K).astype(float)
        q = enum_chain.mcem_conditional(cd, cw, ck, a.astype(np.float64), beta, V * beta)
        rounds = 400_000
        for mode in (1, 2, 3):
            emp = o.frozen_chain(int(inv[t_in]), rounds, mode).astype(float) / rounds
            assert np.abs(emp - q).max() < 0.006, (t_in, mode, emp, q)
        q_sym = enum_chain.mcem_conditional(cd, cw, ck, float(a.mean()), beta, V * beta)
        assert np.abs(q_sym - q).max() > 0.03


def test_log_likelihood_with_alpha_k_normalises():
    """sum over W in [V]^T and Z in [K]^T of exp(LL) = 1 with alpha_k in the
    document part (document lengths fixed)."""
    docs = np.array([0, 0, 1], np.uint32)
    for V, K, a, b in [(2, 2, [0.3, 1.9], 0.4), (2, 3, [2.0, 0.07, 0.6], 0.2)]:
        a = np.array(a, np.float32)
        total = 0.0
        for W in itertools.product(range(V), repeat=3):
            o = oracle.Oracle(np.array(W, np.uint32), docs, V, 2, K, 1, 1.0, b, seed=1)
            o.set_alpha(a)
            o.init()
            _, _, _, inv = o.layout()
            for Z in itertools.product(range(K), repeat=3):
                zcsc = np.empty(3, np.int32)
                zcsc[inv] = Z
                o.set_csc_state(zcsc)
                total += math.exp(o.log_likelihood())
        assert abs(total - 1.0) < 1e-12, (V, K, total)


def test_theta_with_alpha_k():
    """theta_hat_dk = (C_dk + alpha_k) / (L_d + alpha_bar): rows sum to one,
    and theta_hat (L_d + alpha_bar) - alpha_k is the document's count."""
    rng = np.random.default_rng(3)
    T, D, V, K = 400, 12, 30, 5
    w = rng.integers(0, V, T).astype(np.uint32)
    d = rng.integers(0, D, T).astype(np.uint32)
    a = np.array([0.05, 0.4, 1.3, 0.9, 0.2], np.float32)
    o = oracle.Oracle(w, d, V, D, K, 2, 1.0, 0.1, seed=4)
    o.set_alpha(a)
    o.init()
    o.iterate(2)
    th = o.theta()
    z, _ = o.assignments()
    abar = float(np.sum(a.astype(np.float64)))
    for dd in range(D):
        L = int(np.sum(d == dd))
        cnt = np.bincount(z[d == dd], minlength=K)
        assert abs(th[dd].sum() - 1.0) < 1e-12
        assert np.allclose(th[dd] * (L + abar) - a.astype(np.float64), cnt, atol=1e-9)


@pytest.mark.parametrize("case", [
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=2, M=1, alpha=[0.3, 1.7], beta=0.5, n_iter=2),
    dict(words=[0, 1, 1], docs=[0, 0, 0], V=2, K=3, M=2, alpha=[1.2, 0.2, 0.6], beta=0.4, n_iter=1),
])
def test_instant_update_with_alpha_k_matches_enumeration(case):
    w = np.array(case["words"], np.uint32)
    d = np.array(case["docs"], np.uint32)
    K, M, V = case["K"], case["M"], case["V"]
    a = np.array(case["alpha"], np.float32)
    states, pi = enum_chain.instant_distribution_after(list(w), list(d), K, M,
                                                       a.astype(np.float64), case["beta"], V,
                                                       case["n_iter"])
    index = {s: i for i, s in enumerate(states)}
    n = 12000
    counts = np.zeros(len(states))
    for seed in range(n):
        o = oracle.Oracle(w, d, V, int(d.max()) + 1, K, M, 1.0, case["beta"], seed=9000 + seed)
        o.set_alpha(a)
        o.init()
        o.instant_iterate(case["n_iter"])
        z, _ = o.assignments()
        counts[index[tuple(int(x) for x in z)]] += 1
    assert _chi2_p(counts, pi, n) > 1e-4
    # and the enumerated kernel leaves the collapsed posterior with alpha_k invariant
    st, P = enum_chain.instant_iteration_matrix(list(w), list(d), K, M, a.astype(np.float64),
                                                case["beta"], V)
    _, post = enum_chain.collapsed_posterior(list(w), list(d), K, a.astype(np.float64),
                                             case["beta"], V)
    assert np.abs(post @ P - post).max() < 1e-12


def test_set_alpha_validation_and_reset():
    w = np.array([0, 1, 1, 0], np.uint32)
    d = np.array([0, 0, 1, 1], np.uint32)
    o = oracle.Oracle(w, d, 2, 2, 3, 2, 0.5, 0.1, seed=2)
    for bad in ([0.5, 0.0, 1.0], [0.5, -1.0, 1.0], [0.5, np.nan, 1.0], [0.5, np.inf, 1.0]):
        with pytest.raises(RuntimeError):
            o.set_alpha(np.array(bad, np.float32))
    o.set_alpha(np.array([0.5, 0.6, 0.7], np.float32))
    o.set_alpha(None)                      # back to the symmetric alpha
    o.init()
    o.iterate(3)
    ref = oracle.Oracle(w, d, 2, 2, 3, 2, 0.5, 0.1, seed=2)
    ref.init()
    ref.iterate(3)
    assert np.array_equal(o.assignments()[0], ref.assignments()[0])
    assert np.array_equal(o.assignments()[1], ref.assignments()[1])
    with pytest.raises(RuntimeError):      # only before init
        o.set_alpha(np.array([0.5, 0.6, 0.7], np.float32))
