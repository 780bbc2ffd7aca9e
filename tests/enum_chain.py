"""Exact binary64 enumeration of the WarpLDA chain on tiny corpora.

Written from the paper's definitions, independently of the C oracle, to pin it:

* Proposals (Eq. 6), drawn as the two-part mixture of Section 2.2:
    q_doc(k)  = (C_dk + alpha_k) / (L_d + alpha_bar)
    q_word(k) = (C_wk + beta)  / (L_w + K beta)
  (random positioning over a row/column returns topic k with probability
  C_k / L, which gives exactly these laws).
* Acceptance (Eq. 7), with counts frozen for the whole phase (delayed update,
  Section 4.2):
    doc proposal,  judged in the word phase: (C_wc+beta)(C_s+bbar) / ((C_ws+beta)(C_c+bbar))
    word proposal, judged in the doc phase:  (C_dc+alpha_c)(C_s+bbar) / ((C_ds+alpha_s)(C_c+bbar))
  alpha may be a scalar (symmetric prior, alpha_bar = K alpha) or a vector of
  K values alpha_k (asymmetric, alpha_bar = sum_k alpha_k).
* Order (Section 4.4): word phase = judge the pending doc proposals, then draw
  word proposals from the updated column; doc phase = judge the word
  proposals, then draw doc proposals from the updated row.  The first doc
  proposals are drawn from the initial Z.

Because every proposal is drawn independently given the Z it is drawn from,
the assignment vector Z at iteration boundaries is itself a Markov chain on
K^T states, whose transition matrix is built here exactly.
"""
from __future__ import annotations

import itertools
import numpy as np


def _alpha(alpha, K):
    """alpha as K values (a scalar is the symmetric prior)."""
    return np.broadcast_to(np.asarray(alpha, dtype=np.float64), (K,))


def _counts(z, groups, K):
    """Per-group topic histograms (dict group -> array[K])."""
    out = {}
    for g in set(groups):
        out[g] = np.bincount([z[i] for i in range(len(z)) if groups[i] == g],
                             minlength=K).astype(np.float64)
    return out


def _mh_outcome(s0, props_probs, accept, K, M):
    """Distribution of the state after M MH steps whose candidates are iid
    with law props_probs and whose acceptance probability is accept(s, c)."""
    dist = np.zeros(K)
    dist[s0] = 1.0
    for _ in range(M):
        nd = np.zeros(K)
        for s in range(K):
            if dist[s] == 0.0:
                continue
            for c in range(K):
                pc = props_probs[c]
                if pc == 0.0:
                    continue
                a = accept(s, c)
                nd[c] += dist[s] * pc * a
                nd[s] += dist[s] * pc * (1.0 - a)
        dist = nd
    return dist


def phase_matrix(word_ids, doc_ids, K, M, alpha, beta, V, phase, drop_ck=False):
    """K^T x K^T matrix of one phase (the proposal being judged was drawn
    from the same Z the phase starts from)."""
    T = len(word_ids)
    states = list(itertools.product(range(K), repeat=T))
    bbar = V * beta
    av = _alpha(alpha, K)
    abar = av.sum()
    P = np.zeros((len(states), len(states)))
    for si, z in enumerate(states):
        ck = np.bincount(z, minlength=K).astype(np.float64)
        if drop_ck:           # a deliberately wrong rate, for sensitivity checks
            ck = np.zeros(K)
        cw = _counts(z, word_ids, K)
        cd = _counts(z, doc_ids, K)
        per_token = []
        for t in range(T):
            w, d = word_ids[t], doc_ids[t]
            if phase == "word":
                # pending doc proposals, drawn from c_d of this Z
                Ld = cd[d].sum()
                q = (cd[d] + av) / (Ld + abar)
                c_row = cw[w]

                def acc(s, c, c_row=c_row):
                    return min(1.0, (c_row[c] + beta) * (ck[s] + bbar) /
                               ((c_row[s] + beta) * (ck[c] + bbar)))
            else:
                Lw = cw[w].sum()
                q = (cw[w] + beta) / (Lw + K * beta)
                c_row = cd[d]

                def acc(s, c, c_row=c_row):
                    return min(1.0, (c_row[c] + av[c]) * (ck[s] + bbar) /
                               ((c_row[s] + av[s]) * (ck[c] + bbar)))
            per_token.append(_mh_outcome(z[t], q, acc, K, M))
        for sj, z2 in enumerate(states):
            pr = 1.0
            for t in range(T):
                pr *= per_token[t][z2[t]]
                if pr == 0.0:
                    break
            P[si, sj] = pr
    return states, P


def iteration_matrix(word_ids, doc_ids, K, M, alpha, beta, V, drop_ck=False):
    states, Pw = phase_matrix(word_ids, doc_ids, K, M, alpha, beta, V, "word", drop_ck)
    _, Pd = phase_matrix(word_ids, doc_ids, K, M, alpha, beta, V, "doc", drop_ck)
    return states, Pw @ Pd


def distribution_after(word_ids, doc_ids, K, M, alpha, beta, V, n_iter, drop_ck=False):
    """Exact law of Z after n_iter iterations from z ~ iid Uniform(K)."""
    states, P = iteration_matrix(word_ids, doc_ids, K, M, alpha, beta, V, drop_ck)
    pi = np.full(len(states), 1.0 / len(states))
    for _ in range(n_iter):
        pi = pi @ P
    return states, pi


def stationary(word_ids, doc_ids, K, M, alpha, beta, V, iters=5000):
    states, P = iteration_matrix(word_ids, doc_ids, K, M, alpha, beta, V)
    pi = np.full(len(states), 1.0 / len(states))
    for _ in range(iters):
        pi = pi @ P
    return states, pi


def mcem_conditional(cd_row, cw_row, ck, alpha, beta, bbar):
    """q(z = k) of Eq. (5) with frozen counts (token included)."""
    q = (cd_row + alpha) * (cw_row + beta) / (ck + bbar)
    return q / q.sum()


# --------------------------------------------------------------------------
# Fold-in: one new document, C_w and c_k frozen at a trained model's values.
# --------------------------------------------------------------------------
def fold_sweep_matrix(words, K, M, alpha, beta, V, cwk, ck, learned=None, learned_steps=0):
    """K^L x K^L matrix of one fold-in sweep (word step, then doc step with
    optional learned independence steps); the pending doc proposals were drawn
    from the document's current assignments."""
    L = len(words)
    states = list(itertools.product(range(K), repeat=L))
    bbar = V * beta
    cwk = np.asarray(cwk, dtype=np.float64)
    ck = np.asarray(ck, dtype=np.float64)
    index = {s: i for i, s in enumerate(states)}
    # word step
    Pw = np.zeros((len(states), len(states)))
    for si, z in enumerate(states):
        cd = np.bincount(z, minlength=K).astype(np.float64)
        qd = (cd + alpha) / (L + K * alpha)
        per = []
        for t in range(L):
            cw = cwk[words[t]]

            def acc(s, c, cw=cw):
                return min(1.0, (cw[c] + beta) * (ck[s] + bbar) / ((cw[s] + beta) * (ck[c] + bbar)))
            per.append(_mh_outcome(z[t], qd, acc, K, M))
        for sj, z2 in enumerate(states):
            pr = 1.0
            for t in range(L):
                pr *= per[t][z2[t]]
            Pw[si, sj] = pr
    # doc step
    Pd = np.zeros((len(states), len(states)))
    for si, z in enumerate(states):
        cd = np.bincount(z, minlength=K).astype(np.float64)
        per = []
        for t in range(L):
            cw = cwk[words[t]]
            qw = (cw + beta) / (cw.sum() + K * beta)

            def acc(s, c, cd=cd):
                return min(1.0, (cd[c] + alpha) * (ck[s] + bbar) / ((cd[s] + alpha) * (ck[c] + bbar)))
            dist = _mh_outcome(z[t], qw, acc, K, M)
            if learned is not None and learned_steps:
                q = np.asarray(learned, np.float64) / np.sum(learned)
                p = (cd + alpha) * (cw + beta) / (ck + bbar)

                def accl(s, c, p=p, q=q):
                    return min(1.0, p[c] * q[s] / (p[s] * q[c]))
                for _ in range(learned_steps):
                    nd = np.zeros(K)
                    for s0 in range(K):
                        nd += dist[s0] * _mh_outcome(s0, q, accl, K, 1)
                    dist = nd
            per.append(dist)
        for sj, z2 in enumerate(states):
            pr = 1.0
            for t in range(L):
                pr *= per[t][z2[t]]
            Pd[si, sj] = pr
    return states, Pw @ Pd


def fold_distribution(words, K, M, alpha, beta, V, cwk, ck, sweeps, learned=None, learned_steps=0):
    L = len(words)
    states, P = fold_sweep_matrix(words, K, M, alpha, beta, V, cwk, ck, learned, learned_steps)
    if learned is None:
        pi = np.full(len(states), 1.0 / len(states))
    else:
        q = np.asarray(learned, np.float64) / np.sum(learned)
        pi = np.array([np.prod([q[k] for k in s]) for s in states])
    for _ in range(sweeps):
        pi = pi @ P
    return states, pi


# --------------------------------------------------------------------------
# Instant-update (collapsed Gibbs-MH) variant: tokens visited one at a time,
# counts updated as soon as a token moves (Section 6.3's comparison of
# delayed and instant count updates).
# --------------------------------------------------------------------------
def row_order(word_ids, doc_ids):
    """Input indices in the order the scan visits them: documents ascending,
    inside a document by (word, input index) -- ascending canonical column
    position."""
    T = len(word_ids)
    return sorted(range(T), key=lambda i: (doc_ids[i], word_ids[i], i))


def instant_iteration_matrix(word_ids, doc_ids, K, M, alpha, beta, V):
    """K^T x K^T matrix of one instant-update iteration.  For each token in
    scan order, with its own assignment taken out of the counts: M steps with
    q_doc ~ C_dk + alpha judged by the word-side ratio of Eq. (7), then M
    steps with q_word ~ C_wk + beta judged by the document-side ratio."""
    T = len(word_ids)
    states = list(itertools.product(range(K), repeat=T))
    index = {s: i for i, s in enumerate(states)}
    bbar = V * beta
    av = _alpha(alpha, K)
    P = np.eye(len(states))
    for t in row_order(word_ids, doc_ids):
        w, d = word_ids[t], doc_ids[t]
        Pt = np.zeros((len(states), len(states)))
        for si, z in enumerate(states):
            others = [i for i in range(T) if i != t]
            ck = np.bincount([z[i] for i in others], minlength=K).astype(np.float64)
            cd = np.bincount([z[i] for i in others if doc_ids[i] == d], minlength=K).astype(np.float64)
            cw = np.bincount([z[i] for i in others if word_ids[i] == w], minlength=K).astype(np.float64)
            qd = (cd + av) / (cd.sum() + av.sum())
            qw = (cw + beta) / (cw.sum() + K * beta)

            def acc_d(s, c):
                return min(1.0, (cw[c] + beta) * (ck[s] + bbar) / ((cw[s] + beta) * (ck[c] + bbar)))

            def acc_w(s, c):
                return min(1.0, (cd[c] + av[c]) * (ck[s] + bbar) / ((cd[s] + av[s]) * (ck[c] + bbar)))
            dist = _mh_outcome(z[t], qd, acc_d, K, M)
            nd = np.zeros(K)
            for s0 in range(K):
                if dist[s0]:
                    nd += dist[s0] * _mh_outcome(s0, qw, acc_w, K, M)
            for k in range(K):
                z2 = list(z)
                z2[t] = k
                Pt[si, index[tuple(z2)]] += nd[k]
        P = P @ Pt
    return states, P


def instant_distribution_after(word_ids, doc_ids, K, M, alpha, beta, V, n_iter):
    """Exact law of Z after n_iter instant-update iterations from z ~ iid Uniform(K)."""
    states, P = instant_iteration_matrix(word_ids, doc_ids, K, M, alpha, beta, V)
    pi = np.full(len(states), 1.0 / len(states))
    for _ in range(n_iter):
        pi = pi @ P
    return states, pi


def collapsed_posterior(word_ids, doc_ids, K, alpha, beta, V):
    """p(Z | W) of Eq. (1), by enumeration: proportional to the product over
    documents of prod_k Gamma(alpha_k + C_dk) and over topics of
    prod_w Gamma(beta + C_wk) / Gamma(V beta + C_k)."""
    from math import lgamma
    T = len(word_ids)
    states = list(itertools.product(range(K), repeat=T))
    av = _alpha(alpha, K)
    logp = np.zeros(len(states))
    for si, z in enumerate(states):
        lp = 0.0
        for d in set(doc_ids):
            c = np.bincount([z[i] for i in range(T) if doc_ids[i] == d], minlength=K)
            lp += sum(lgamma(av[k] + x) for k, x in enumerate(c))
        for w in set(word_ids):
            c = np.bincount([z[i] for i in range(T) if word_ids[i] == w], minlength=K)
            lp += sum(lgamma(beta + x) for x in c)
        ck = np.bincount(list(z), minlength=K)
        lp -= sum(lgamma(V * beta + x) for x in ck)
        logp[si] = lp
    p = np.exp(logp - logp.max())
    return states, p / p.sum()
