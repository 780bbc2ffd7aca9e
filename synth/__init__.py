"""Seeded synthetic corpora for the WarpLDA sweep.

This module only draws inputs.  It holds none of the sampler's arithmetic and
is shared by the tests, the benchmark and the smoke check, which feed the same
token lists to the CPU oracle and to the HIP library.

Corpus shapes follow the dataset table of the paper (Section 6.1, Table 3:
NYTimes D=300K, T=100M, V=102K; PubMed D=8.2M, T=738M, V=141K; ClueWeb12
V=1M).  The datasets themselves are not available, so these generators stand in
for them:

* ``lda_corpus``    - the LDA generative process of Section 2.1 (theta_d ~
  Dir(alpha), phi_k ~ Dir(beta), z ~ Mult(theta_d), w ~ Mult(phi_z)) with
  Poisson document lengths.
* ``zipf_corpus``   - iid words from a truncated Zipf(s) law over V ranks
  (ranks mapped to word ids through a seeded permutation), document lengths
  round(lognormal) with the given distribution *mean* (mu = ln m - sigma^2/2),
  clipped to >= 1.

Every array is uint32; tokens are emitted document by document, but nothing
downstream relies on that order.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CORPUS_SEED_BASE = 20151028


@dataclasses.dataclass
class Corpus:
    word_ids: np.ndarray          # uint32[T]
    doc_ids: np.ndarray           # uint32[T]
    V: int
    D: int
    true_z: np.ndarray | None = None   # int32[T] for LDA-generated corpora

    @property
    def T(self) -> int:
        return int(self.word_ids.shape[0])


def _lognormal_lengths(rng, D, mean, sigma, lo=1, hi=None):
    mu = np.log(mean) - 0.5 * sigma * sigma
    L = np.rint(rng.lognormal(mu, sigma, size=D)).astype(np.int64)
    L = np.maximum(L, lo)
    if hi is not None:
        L = np.minimum(L, hi)
    return L


def zipf_corpus(D: int, V: int, s: float, mean_len: float, sigma: float,
                seed: int, chunk: int = 1 << 24, n_docs: int | None = None) -> Corpus:
    """iid Zipf(s) words over V ranks, lognormal document lengths.  With
    n_docs, only the first n_docs documents of that same corpus (its document
    prefix: the lengths of all D documents are drawn, then the words of the
    first n_docs in order, so every token equals the full corpus's)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = _lognormal_lengths(rng, D, mean_len, sigma)
    if n_docs is not None:
        D = min(D, int(n_docs))
        lengths = lengths[:D]
    T = int(lengths.sum())
    if T >= 1 << 32:
        raise ValueError("corpus too large for 32-bit token indices")
    w = np.arange(1, V + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rank_to_word = rng.permutation(V).astype(np.uint32)
    word_ids = np.empty(T, dtype=np.uint32)

    def fill(lo, u):   # inverse CDF of one chunk (numpy releases the GIL here)
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, V - 1, out=r)
        word_ids[lo:lo + len(u)] = rank_to_word[r]

    # the uniforms are drawn in order from the one generator, so the corpus
    # does not depend on how many threads convert them
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        pending = []
        for lo in range(0, T, chunk):
            pending.append(ex.submit(fill, lo, rng.random(min(T, lo + chunk) - lo)))
            if len(pending) >= 2 * workers:
                pending.pop(0).result()
        for f in pending:
            f.result()
    doc_ids = np.repeat(np.arange(D, dtype=np.uint32), lengths)
    return Corpus(word_ids, doc_ids, V, D)


def lda_corpus(D: int, V: int, K: int, mean_len: float, alpha: float,
               beta: float, seed: int) -> Corpus:
    """The LDA generative process with Poisson(mean_len) document lengths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = rng.dirichlet(np.full(V, beta), size=K)          # K x V
    theta = rng.dirichlet(np.full(K, alpha), size=D)       # D x K
    lengths = np.maximum(rng.poisson(mean_len, size=D), 1)
    T = int(lengths.sum())
    doc_ids = np.repeat(np.arange(D, dtype=np.uint32), lengths)
    word_ids = np.empty(T, dtype=np.uint32)
    true_z = np.empty(T, dtype=np.int32)
    cphi = np.cumsum(phi, axis=1)
    cphi /= cphi[:, -1:]
    ctheta = np.cumsum(theta, axis=1)
    ctheta /= ctheta[:, -1:]
    pos = 0
    for d in range(D):
        n = int(lengths[d])
        z = np.searchsorted(ctheta[d], rng.random(n), side="right")
        np.minimum(z, K - 1, out=z)
        u = rng.random(n)
        wv = np.empty(n, dtype=np.int64)
        for k in np.unique(z):
            m = z == k
            wv[m] = np.searchsorted(cphi[k], u[m], side="right")
        np.minimum(wv, V - 1, out=wv)
        word_ids[pos:pos + n] = wv
        true_z[pos:pos + n] = z
        pos += n
    return Corpus(word_ids, doc_ids, V, D, true_z)


def random_corpus(T: int, V: int, D: int, seed: int) -> Corpus:
    """Uniform word and doc ids (small edge-case corpora for the tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return Corpus(rng.integers(0, V, T, dtype=np.uint32),
                  rng.integers(0, D, T, dtype=np.uint32), V, D)


# --------------------------------------------------------------------------
# Named workloads (sizes from the paper's dataset table; fit settings from the
# paper's experimental setup: alpha = 50/K, beta = 0.01).
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    K: int
    M: int
    alpha: float
    beta: float
    iters: int
    make: object          # () -> Corpus


WORKLOADS = {
    "tiny-lda-k16": Workload(
        "tiny-lda-k16", K=16, M=2, alpha=50.0 / 16, beta=0.01, iters=50,
        make=lambda: lda_corpus(1000, 2000, 16, 100.0, 50.0 / 16, 0.01,
                                CORPUS_SEED_BASE + 0)),
    "nytimes-shape-k1e3": Workload(
        "nytimes-shape-k1e3", K=1000, M=2, alpha=0.05, beta=0.01, iters=100,
        make=lambda: zipf_corpus(300_000, 100_000, 1.0, 330.0, 0.8,
                                 CORPUS_SEED_BASE + 1)),
    "pubmed-shape-k1e4": Workload(
        "pubmed-shape-k1e4", K=10_000, M=4, alpha=0.005, beta=0.01, iters=50,
        make=lambda n_docs=None: zipf_corpus(8_000_000, 140_000, 1.05, 90.0, 0.7,
                                             CORPUS_SEED_BASE + 2, n_docs=n_docs)),
    "clueweb-share-k1e6": Workload(
        "clueweb-share-k1e6", K=1_000_000, M=2, alpha=0.01, beta=0.01, iters=20,
        make=lambda n_docs=None: zipf_corpus(20_000_000, 1_000_000, 1.1, 100.0, 1.0,
                                             CORPUS_SEED_BASE + 3, n_docs=n_docs)),
}


WORKLOADS["nytimes-shape-topical-k1e3"] = Workload(
    "nytimes-shape-topical-k1e3", K=1000, M=2, alpha=0.05, beta=0.01, iters=100,
    make=lambda: topical_zipf_corpus(300_000, 100_000, 1000, 1.0, 330.0, 0.8, 0.05, 2.0,
                                     CORPUS_SEED_BASE + 11))


def doc_prefix(c: Corpus, n_docs: int) -> Corpus:
    """The tokens of documents [0, n_docs) (the generators emit docs in order)."""
    n = int(np.searchsorted(c.doc_ids, n_docs, side="left"))
    tz = None if c.true_z is None else c.true_z[:n]
    return Corpus(c.word_ids[:n], c.doc_ids[:n], c.V, n_docs, tz)


def encoder_init_weights(buckets: int, hidden: int, K: int, seed: int, w1_std: float = 0.25):
    """Seeded He-style initial weights of the proposal encoder (float32):
    [W1 (buckets x hidden), b1, W2 (hidden x hidden), b2, W3 (hidden x K), b3].
    The first layer averages ~L rows (features tf/L), so its scale is set
    separately (w1_std)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [
        (rng.standard_normal((buckets, hidden)) * w1_std).astype(np.float32),
        np.zeros(hidden, np.float32),
        (rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)).astype(np.float32),
        np.zeros(hidden, np.float32),
        (rng.standard_normal((hidden, K)) * np.sqrt(1.0 / hidden)).astype(np.float32),
        np.zeros(K, np.float32),
    ]


def docs_from_model(word_ids, z, V: int, K: int, alpha: float, beta: float, n_docs: int,
                    seed: int, mean_len_log: float = 5.76, sigma: float = 0.89,
                    lo: int = 20, hi: int = 5000):
    """New documents drawn from a fitted model: theta ~ Dir(alpha), z ~ theta,
    w ~ phi_z with phi_k proportional to C_wk + beta (the counts of the given
    assignments).  Lengths round(lognormal(mean_len_log, sigma)) clipped to
    [lo, hi] (median ~316 for the defaults).  Each document's tokens are split
    50/50 at random into an observed part and a held-out part.
    Returns (docptr, words, hoptr, held_out_words), uint64/uint32 arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cw = np.bincount(np.asarray(word_ids, np.int64) * K + np.asarray(z, np.int64),
                     minlength=V * K).reshape(V, K)
    lens = np.clip(np.rint(rng.lognormal(mean_len_log, sigma, n_docs)), lo, hi).astype(np.int64)
    theta = rng.dirichlet(np.full(K, alpha), size=n_docs)
    ctheta = np.cumsum(theta, axis=1)
    ctheta /= ctheta[:, -1:]
    T = int(lens.sum())
    topics = np.empty(T, np.int64)
    pos = 0
    for d in range(n_docs):
        t = np.searchsorted(ctheta[d], rng.random(lens[d]), side="right")
        topics[pos:pos + lens[d]] = np.minimum(t, K - 1)
        pos += lens[d]
    words = np.empty(T, np.uint32)
    u = rng.random(T)
    for k in np.unique(topics):
        m = topics == k
        cdf = np.cumsum(cw[:, k] + beta)
        words[m] = np.minimum(np.searchsorted(cdf / cdf[-1], u[m], side="right"), V - 1)
    obs, held, op, hp = [], [], [0], [0]
    pos = 0
    for d in range(n_docs):
        w = words[pos:pos + lens[d]][rng.permutation(lens[d])]
        pos += lens[d]
        h = lens[d] // 2
        obs.append(w[h:])
        held.append(w[:h])
        op.append(op[-1] + len(w) - h)
        hp.append(hp[-1] + h)
    return (np.array(op, np.uint64), np.concatenate(obs), np.array(hp, np.uint64),
            np.concatenate(held))


def poisson_arrivals(n: int, rate: float, seed: int):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))


def topical_zipf_corpus(D: int, V: int, K: int, s: float, mean_len: float, sigma: float,
                        alpha: float, tilt: float, seed: int) -> Corpus:
    """LDA-generated corpus with Zipf-shaped topics: phi_k(w) proportional to
    r(w)^-s * exp(tilt * e_kw), e_kw ~ N(0, 1), so every topic keeps the
    Zipf(s) profile of word frequencies but favours its own words; theta_d ~
    Dir(alpha); lognormal document lengths as in zipf_corpus."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = _lognormal_lengths(rng, D, mean_len, sigma)
    T = int(lengths.sum())
    base = np.arange(1, V + 1, dtype=np.float64) ** (-s)
    rank_to_word = rng.permutation(V).astype(np.uint32)
    topics = np.empty(T, np.int32)
    pos = 0
    for d0 in range(0, D, 8192):            # topic counts per document, in chunks
        d1 = min(D, d0 + 8192)
        theta = rng.dirichlet(np.full(K, alpha), size=d1 - d0)
        counts = rng.multinomial(lengths[d0:d1], theta)
        n = int(lengths[d0:d1].sum())
        topics[pos:pos + n] = np.repeat(np.tile(np.arange(K, dtype=np.int32), d1 - d0),
                                        counts.ravel())
        pos += n
    word_ids = np.empty(T, np.uint32)
    u = rng.random(T)
    order = np.argsort(topics, kind="stable")
    bounds = np.searchsorted(topics[order], np.arange(K + 1))
    for k in range(K):
        sel = order[bounds[k]:bounds[k + 1]]
        if len(sel) == 0:
            continue
        phi = base * np.exp(tilt * rng.standard_normal(V))
        cdf = np.cumsum(phi)
        r = np.minimum(np.searchsorted(cdf / cdf[-1], u[sel], side="right"), V - 1)
        word_ids[sel] = rank_to_word[r]
    doc_ids = np.repeat(np.arange(D, dtype=np.uint32), lengths)
    return Corpus(word_ids, doc_ids, V, D, topics)


def _polya_topics(rng, lengths, K: int, alpha: float) -> np.ndarray:
    """Topic assignments of documents with theta_d ~ Dir(alpha) integrated
    out (the Dirichlet-multinomial predictive rule): token n of a document
    copies the topic of a uniformly chosen earlier token with probability
    n / (n + K alpha), else takes a uniform topic, so P(z_n = k | z_<n) =
    (C_k + alpha) / (n + K alpha).  Vectorised over documents, position by
    position."""
    lengths = np.asarray(lengths, np.int64)
    off = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    by_len = np.argsort(-lengths, kind="stable")
    sorted_len = lengths[by_len]
    topics = np.empty(int(lengths.sum()), np.int32)
    for n in range(int(lengths.max()) if len(lengths) else 0):
        m = int(np.searchsorted(-sorted_len, -n, side="left"))   # documents longer than n
        base = off[by_len[:m]]
        u, v = rng.random(m), rng.random(m)
        fresh = rng.integers(0, K, m, dtype=np.int32)
        if n == 0:
            topics[base] = fresh
            continue
        copy = u * (n + K * alpha) < n
        src = base + np.minimum((v * n).astype(np.int64), n - 1)
        topics[base + n] = np.where(copy, topics[src], fresh)
    return topics


def lda_sparse_corpus(D: int, V: int, K: int, mean_len: float, sigma: float, alpha: float,
                      beta_topic: float, seed: int) -> Corpus:
    """The LDA generative process of Section 2.1 with sparse topics:
    phi_k ~ Dir(beta_topic) over the V words, theta_d ~ Dir(alpha), z ~ theta_d
    (drawn with theta_d integrated out, _polya_topics), w ~ phi_z, with
    lognormal document lengths as in zipf_corpus.  Small
    beta_topic gives topics that own disjoint sets of words, so a document's
    topics can be read off its words."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = _lognormal_lengths(rng, D, mean_len, sigma)
    T = int(lengths.sum())
    topics = _polya_topics(rng, lengths, K, alpha)
    word_ids = np.empty(T, np.uint32)
    u = rng.random(T)
    # tokens grouped by topic (a radix sort when the topics fit 16 bits)
    order = np.argsort(topics.astype(np.int16) if K <= 32767 else topics, kind="stable")
    bounds = np.searchsorted(topics[order], np.arange(K + 1))

    def fill(k, g):   # words of topic k by inverse CDF (numpy releases the GIL)
        sel = order[bounds[k]:bounds[k + 1]]
        if len(sel) == 0 or g.sum() <= 0:
            return
        cdf = np.cumsum(g)
        word_ids[sel] = np.minimum(np.searchsorted(cdf / cdf[-1], u[sel], side="right"), V - 1)

    # phi_k ~ Dir(beta_topic) by normalised gammas, drawn in topic order from
    # the one generator (so the corpus does not depend on the thread count)
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        pending = []
        for k in range(K):
            pending.append(ex.submit(fill, k, rng.standard_gamma(beta_topic, V)))
            if len(pending) >= 2 * workers:
                pending.pop(0).result()
        for f in pending:
            f.result()
    doc_ids = np.repeat(np.arange(D, dtype=np.uint32), lengths)
    return Corpus(word_ids, doc_ids, V, D, topics)


# NYTimes-shaped LDA corpus with sparse topics (phi_k ~ Dir(0.01) over 100k
# words) and documents of few topics (theta_d ~ Dir(0.01), about 35 topics in
# a 330-token document), fitted with the paper's alpha = 50/K: the model the
# fold-in experiments freeze
WORKLOADS["nytimes-shape-lda-k1e3"] = Workload(
    "nytimes-shape-lda-k1e3", K=1000, M=2, alpha=0.05, beta=0.01, iters=100,
    make=lambda: lda_sparse_corpus(300_000, 100_000, 1000, 330.0, 0.8, 0.01, 0.01,
                                   CORPUS_SEED_BASE + 12))
