"""Exact binary64 enumeration of the WarpLDA chain on tiny corpora.

Written from the paper's definitions, independently of the C oracle, to pin it:

* Proposals (Eq. 6), drawn as the two-part mixture of Section 2.2:
    q_doc(k)  = (C_dk + alpha) / (L_d + K alpha)
    q_word(k) = (C_wk + beta)  / (L_w + K beta)
  (random positioning over a row/column returns topic k with probability
  C_k / L, which gives exactly these laws).
* Acceptance (Eq. 7), with counts frozen for the whole phase (delayed update,
  Section 4.2):
    doc proposal,  judged in the word phase: (C_wc+beta)(C_s+bbar) / ((C_ws+beta)(C_c+bbar))
    word proposal, judged in the doc phase:  (C_dc+alpha)(C_s+bbar) / ((C_ds+alpha)(C_c+bbar))
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
                q = (cd[d] + alpha) / (Ld + K * alpha)
                c_row = cw[w]

                def acc(s, c, c_row=c_row):
                    return min(1.0, (c_row[c] + beta) * (ck[s] + bbar) /
                               ((c_row[s] + beta) * (ck[c] + bbar)))
            else:
                Lw = cw[w].sum()
                q = (cw[w] + beta) / (Lw + K * beta)
                c_row = cd[d]

                def acc(s, c, c_row=c_row):
                    return min(1.0, (c_row[c] + alpha) * (ck[s] + bbar) /
                               ((c_row[s] + alpha) * (ck[c] + bbar)))
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
