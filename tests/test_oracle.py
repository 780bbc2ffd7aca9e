"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: every expected value comes from
a closed form, an exact enumeration written separately from the paper's
definitions (enum_chain.py), an independent Philox implementation (rocRAND),
or an invariant of the model.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
import enum_chain


@pytest.fixture(scope="session", autouse=True)
def _built():
    oracle.build(force=False)


# --------------------------------------------------------------------------
# Philox4x32-10: the oracle's copy against rocRAND's, run on the host.
# --------------------------------------------------------------------------
ROCRAND_PROBE = r"""
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
// ten_rounds() is a protected member: reach it through a derived class.
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    Probe eng;
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint4 r = eng.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand():
    """P6: the oracle's Philox4x32-10 equals rocRAND's on 2000 key/counters."""
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "probe.hip")
        exe = os.path.join(td, "probe")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-O1", "--offload-arch=gfx950", src, "-o", exe],
                              stderr=subprocess.DEVNULL)
        rng = np.random.default_rng(5)
        kc = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
        kc[:5] = 0
        kc[5] = 2**32 - 1
        kc[6, 2:] = [3, 7, (2 << 16) | 1, 0]
        inp = "\n".join(" ".join(str(int(x)) for x in row) for row in kc) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                             check=True).stdout.split("\n")
        for row, line in zip(kc, out):
            want = [int(x) for x in line.split()]
            got = oracle.philox(row[:2], row[2:]).tolist()
            assert got == want, (row, got, want)


# --------------------------------------------------------------------------
# Layout (Section 5.2): columns sorted by doc id, rows point into them.
# --------------------------------------------------------------------------
def test_layout_definition():
    c = synth.random_corpus(500, 37, 23, seed=3)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=4, M=1, alpha=0.1, beta=0.1)
    colptr, rowptr, row, inv = o.layout()
    order = np.lexsort((np.arange(c.T), c.doc_ids, c.word_ids))
    expect_inv = np.empty(c.T, dtype=np.int64)
    expect_inv[order] = np.arange(c.T)
    assert np.array_equal(inv, expect_inv)
    assert np.array_equal(colptr, np.concatenate([[0], np.cumsum(np.bincount(c.word_ids, minlength=c.V))]))
    assert np.array_equal(rowptr, np.concatenate([[0], np.cumsum(np.bincount(c.doc_ids, minlength=c.D))]))
    doc_csc = c.doc_ids[order]
    for d in range(c.D):
        r = row[rowptr[d]:rowptr[d + 1]]
        assert np.all(np.diff(r.astype(np.int64)) > 0)
        assert np.all(doc_csc[r] == d)


def test_rejects_invalid_inputs():
    w = np.array([0, 1], dtype=np.uint32)
    d = np.array([0, 0], dtype=np.uint32)
    for kw in [dict(K=0), dict(M=0), dict(M=5), dict(alpha=0.0), dict(beta=-1.0)]:
        args = dict(V=2, D=1, K=2, M=1, alpha=0.1, beta=0.1)
        args.update(kw)
        with pytest.raises(ValueError):
            oracle.Oracle(w, d, **args)
    with pytest.raises(ValueError):      # word id out of range
        oracle.Oracle(w, d, V=1, D=1, K=2, M=1, alpha=0.1, beta=0.1)


# --------------------------------------------------------------------------
# P1: count invariants after every phase.
# --------------------------------------------------------------------------
def test_count_invariants_every_phase():
    c = synth.random_corpus(3000, 50, 40, seed=11)
    K = 7
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=K, M=2, alpha=0.3, beta=0.05, seed=9)
    o.init()
    for phase in range(10):
        (o.word_phase if phase % 2 == 0 else o.doc_phase)()
        z, p = o.assignments()
        ck = o.topic_counts()
        assert ck.sum() == c.T
        assert np.array_equal(ck, np.bincount(z, minlength=K))
        assert z.min() >= 0 and z.max() < K and p.min() >= 0 and p.max() < K
        cdk = np.zeros((c.D, K), np.int64)
        np.add.at(cdk, (c.doc_ids, z), 1)
        cwk = np.zeros((c.V, K), np.int64)
        np.add.at(cwk, (c.word_ids, z), 1)
        assert np.array_equal(cdk.sum(1), np.bincount(c.doc_ids, minlength=c.D))
        assert np.array_equal(cwk.sum(1), np.bincount(c.word_ids, minlength=c.V))
        assert np.array_equal(cwk.sum(0), ck)


def test_phase_order_enforced():
    c = synth.random_corpus(20, 3, 2, seed=1)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=3, M=1, alpha=0.1, beta=0.1)
    with pytest.raises(RuntimeError):
        o.word_phase()                 # before init
    o.init()
    with pytest.raises(RuntimeError):
        o.doc_phase()                  # word phase must come first


# --------------------------------------------------------------------------
# P4: D = V = 1 with alpha = beta reduces to a Wright-Fisher chain.
# --------------------------------------------------------------------------
def test_wright_fisher_special_case():
    """With one document, one word and alpha = beta, both acceptance ratios
    of Eq. (7) are exactly 1 (every MH step accepts), and each phase redraws
    every z iid from (C_k + alpha) / (T + K alpha).  For T = K = 2 the
    two-state chain (equal / split) gives P(z1 == z2) = 1 / (3 - 2a) with
    a = ((2+alpha)^2 + alpha^2) / (4 (1+alpha)^2); 4/7 at alpha = 1."""
    alpha = 1.0
    a = ((2 + alpha) ** 2 + alpha ** 2) / (4 * (1 + alpha) ** 2)
    p_eq = 1.0 / (3 - 2 * a)
    assert abs(p_eq - 4.0 / 7.0) < 1e-15
    w = np.zeros(2, np.uint32)
    d = np.zeros(2, np.uint32)
    n_chains, eq = 6000, 0
    for seed in range(n_chains):
        o = oracle.Oracle(w, d, V=1, D=1, K=2, M=2, alpha=alpha, beta=alpha, seed=seed)
        o.init()
        for _ in range(4):
            o.word_phase()
            assert o.accepted(oracle.PH_WORD) == 2 * 2
            o.doc_phase()
            assert o.accepted(oracle.PH_DOC) == 2 * 2
        z, _ = o.assignments()
        eq += int(z[0] == z[1])
    se = math.sqrt(p_eq * (1 - p_eq) / n_chains)
    assert abs(eq / n_chains - p_eq) < 4 * se, (eq / n_chains, p_eq)
    # the collapsed posterior would give (alpha+1)/(2 alpha+1) = 2/3: the
    # delayed-update chain does not target it, and the test can tell.
    assert abs(2.0 / 3.0 - p_eq) > 10 * se


# --------------------------------------------------------------------------
# P3: exact enumeration of the delayed-update chain.
# --------------------------------------------------------------------------
def _chi2_ok(counts, probs, n, min_expected=5.0):
    from scipy import stats
    mask = probs * n >= min_expected
    obs = np.append(counts[mask], counts[~mask].sum())
    exp = np.append(probs[mask] * n, probs[~mask].sum() * n)
    if exp[-1] < 1e-9:
        obs, exp = obs[:-1], exp[:-1]
    chi2 = ((obs - exp) ** 2 / exp).sum()
    return stats.chi2.sf(chi2, len(obs) - 1)


@pytest.mark.parametrize("case", [
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=1, alpha=0.7, beta=0.4, n_iter=1),
    dict(words=[0, 1, 0], docs=[0, 0, 1], V=2, K=3, M=2, alpha=0.7, beta=0.4, n_iter=2),
    dict(words=[0, 0, 1, 1], docs=[0, 1, 0, 1], V=2, K=2, M=1, alpha=0.3, beta=0.9, n_iter=3),
    dict(words=[0, 1, 2, 1], docs=[0, 0, 0, 1], V=3, K=3, M=1, alpha=0.5, beta=0.2, n_iter=2),
    # L_w > K: word 0's proposals come from the inverse CDF of its updated
    # counts (Section 5.4's words, whose proposal is drawn from a table over
    # c_w); the law is that of random positioning
    dict(words=[0, 0, 0, 1], docs=[0, 1, 0, 1], V=2, K=2, M=1, alpha=0.6, beta=0.3, n_iter=2),
    dict(words=[0, 0, 0, 1, 0], docs=[0, 1, 0, 1, 1], V=2, K=2, M=2, alpha=0.4, beta=0.7, n_iter=2),
    # the boundary: L_w = K (random positioning) and L_w = K + 1 (inverse CDF)
    dict(words=[0, 0, 0, 1], docs=[0, 1, 0, 1], V=2, K=3, M=1, alpha=0.5, beta=0.25, n_iter=2),
    dict(words=[0, 0, 0, 0, 1], docs=[0, 1, 0, 1, 1], V=2, K=3, M=1, alpha=0.5, beta=0.25, n_iter=2),
])
def test_chain_law_matches_enumeration(case):
    """The law of Z after n iterations from the oracle's init equals the exact
    enumeration (chi-square over independently seeded chains)."""
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
        o = oracle.Oracle(w, d, V, D, K, M, case["alpha"], case["beta"], seed=1000 + seed)
        o.init()
        o.iterate(case["n_iter"])
        z, _ = o.assignments()
        counts[index[tuple(int(x) for x in z)]] += 1
    p = _chi2_ok(counts, pi, n)
    assert p > 1e-4, p


def test_enumeration_is_sensitive_to_a_wrong_rate():
    """Sanity of the pin itself: a plausible slip (dropping the c_k factor of
    Eq. 7) changes the enumerated law by far more than the chi-square test
    above can miss at n = 12000."""
    w, d = [0, 1, 0], [0, 0, 1]
    _, right = enum_chain.distribution_after(w, d, 3, 2, 0.7, 0.4, 2, 2)
    _, wrong = enum_chain.distribution_after(w, d, 3, 2, 0.7, 0.4, 2, 2, drop_ck=True)
    # total-variation gap vs the ~sqrt(states/n) resolution of the test
    assert 0.5 * np.abs(right - wrong).sum() > 4 * np.sqrt(len(right) / 12000)


# --------------------------------------------------------------------------
# P2: per-token stationarity of the MH kernels against Eq. (5).
# --------------------------------------------------------------------------
def test_frozen_count_chain_targets_eq5():
    rng = np.random.default_rng(4)
    T = 30
    w = rng.integers(0, 4, T).astype(np.uint32)
    d = rng.integers(0, 3, T).astype(np.uint32)
    K, alpha, beta, V = 3, 0.6, 0.3, 4
    o = oracle.Oracle(w, d, V, 3, K, 2, alpha, beta, seed=77)
    zin = rng.integers(0, K, T).astype(np.int32)
    zin[:12] = 0                      # uneven topic totals so c_k matters
    o.init()
    # put zin into the sampler (CSC order) via the layout
    _, _, _, inv = o.layout()
    zcsc = np.empty(T, np.int32)
    zcsc[inv] = zin
    o.set_csc_state(zcsc)
    ck = np.bincount(zin, minlength=K).astype(float)
    for t_in in [0, 17, 29]:
        cd = np.bincount(zin[d == d[t_in]], minlength=K).astype(float)
        cw = np.bincount(zin[w == w[t_in]], minlength=K).astype(float)
        q = enum_chain.mcem_conditional(cd, cw, ck, alpha, beta, V * beta)
        rounds = 400_000
        for mode in (1, 2, 3):
            hist = o.frozen_chain(int(inv[t_in]), rounds, mode).astype(float)
            emp = hist / rounds
            assert np.abs(emp - q).max() < 0.006, (t_in, mode, emp, q)
        # a target without the 1/(C_k + bbar) factor would be far away
        q_bad = (cd + alpha) * (cw + beta)
        q_bad /= q_bad.sum()
        assert np.abs(q_bad - q).max() > 0.03


# --------------------------------------------------------------------------
# P5: log joint likelihood of Section 6.1.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("K,V", [(2, 3), (5, 7), (1000, 100000)])
def test_ll_single_token(K, V):
    """T = 1: every Gamma ratio collapses and LL = -log K - log V."""
    ll = oracle.log_joint([V - 1], [0], [K - 1], V, 1, K, 50.0 / K, 0.01)
    assert abs(ll - (-math.log(K) - math.log(V))) < 1e-9


def test_ll_normalises():
    """sum over all W in [V]^T and Z in [K]^T of exp(LL) = 1 (doc lengths fixed)."""
    import itertools
    docs = [0, 0, 1]
    for V, K, a, b in [(2, 2, 0.5, 0.3), (2, 3, 1.7, 0.05), (3, 2, 0.1, 2.0)]:
        total = 0.0
        for W in itertools.product(range(V), repeat=3):
            for Z in itertools.product(range(K), repeat=3):
                total += math.exp(oracle.log_joint(W, docs, Z, V, 2, K, a, b))
        assert abs(total - 1.0) < 1e-12, (V, K, total)


def test_sampler_ll_equals_log_joint():
    c = synth.random_corpus(2000, 30, 25, seed=2)
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=6, M=2, alpha=0.2, beta=0.03)
    o.init()
    o.iterate(3)
    z, _ = o.assignments()
    ref = oracle.log_joint(c.word_ids, c.doc_ids, z, c.V, c.D, 6, 0.2, 0.03)
    assert abs(o.log_likelihood() - ref) <= 1e-12 * abs(ref)


# --------------------------------------------------------------------------
# P8: order independence and checkpoint/resume.
# --------------------------------------------------------------------------
def test_visit_order_does_not_matter():
    c = synth.random_corpus(4000, 60, 50, seed=21)
    a = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=9, M=2, alpha=0.4, beta=0.02, seed=5)
    b = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K=9, M=2, alpha=0.4, beta=0.02, seed=5)
    b.set_visit_reversed(True)
    for o in (a, b):
        o.init()
        o.iterate(4)
    za, pa = a.assignments()
    zb, pb = b.assignments()
    assert np.array_equal(za, zb) and np.array_equal(pa, pb)


def test_checkpoint_resume_bit_identical():
    c = synth.random_corpus(3000, 40, 30, seed=8)
    args = (c.word_ids, c.doc_ids, c.V, c.D, 5, 2, 0.3, 0.05, 3)
    ref = oracle.Oracle(*args)
    ref.init()
    ref.iterate(2)
    ref.word_phase()
    blob = ref.save_state()
    ref.doc_phase()
    ref.iterate(2)
    other = oracle.Oracle(*args)
    other.load_state(blob)
    other.doc_phase()
    other.iterate(2)
    assert np.array_equal(ref.assignments()[0], other.assignments()[0])
    assert np.array_equal(ref.assignments()[1], other.assignments()[1])
    assert ref.iteration == other.iteration == 5


# --------------------------------------------------------------------------
# P7: sanity on the LDA-generated corpus (parity unpinned numerically).
# --------------------------------------------------------------------------
def test_tiny_lda_ll_rises():
    c = synth.doc_prefix(synth.WORKLOADS["tiny-lda-k16"].make(), 200)
    K = 16
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, 2, 50.0 / K, 0.01, seed=1)
    o.init()
    ll0 = o.log_likelihood()
    o.iterate(30)
    ll30 = o.log_likelihood()
    truth = oracle.log_joint(c.word_ids, c.doc_ids, c.true_z, c.V, c.D, K, 50.0 / K, 0.01)
    assert ll30 > ll0 + 0.1 * abs(ll0 - truth)
