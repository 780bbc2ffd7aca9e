"""One phase of one column or one row of a large corpus, on the oracle.

A word phase treats every column on its own given the phase-start state (z
and the pending doc proposals of its tokens) and the global c_k; a doc phase
does the same for every row.  So the oracle, loaded with a corpus that is one
column (row) of a larger one, set to the larger corpus's state and told where
the column (row) starts in the larger corpus's canonical order (the Philox
token index), reproduces that column's (row's) outcome exactly.  This lets
the tests check sampled columns and rows of corpora far too large for the
whole oracle."""
import numpy as np

import oracle


def column_order(word_ids, doc_ids, w):
    """Input indices of word w's tokens in canonical column order (by
    document, then input index)."""
    idx = np.nonzero(word_ids == w)[0]
    return idx[np.lexsort((idx, doc_ids[idx]))]


def row_order(word_ids, doc_ids, d):
    """Input indices of document d's tokens in canonical row order (ascending
    column-major position: by word, then input index)."""
    idx = np.nonzero(doc_ids == d)[0]
    return idx[np.lexsort((idx, word_ids[idx]))]


def column_phase(V, K, M, alpha, beta, seed, iteration, csc_off, doc_ids_col, z_pre, p_pre, ck):
    """The word phase of one column: its tokens' documents (in column order),
    their phase-start z and pending doc proposals (M x n), the global c_k.
    Returns the column's new z and word proposals, in column order."""
    n = len(z_pre)
    _, d = np.unique(doc_ids_col, return_inverse=True)          # documents by rank
    o = oracle.Oracle(np.zeros(n, np.uint32), d.astype(np.uint32), V, int(d.max()) + 1, K, M,
                      alpha, beta, seed=seed)
    o.init()
    o.set_csc_state(np.asarray(z_pre, np.int32), np.asarray(p_pre, np.int32))
    o.set_token_offsets(csc_off, 0)
    o.set_phase_state(ck, oracle.PH_WORD, iteration)
    o.word_phase()
    return o.csc()


def row_phase(V, K, M, alpha, beta, seed, iteration, csr_off, word_ids_row, z_pre, p_pre, ck):
    """The doc phase of one row: its tokens' words (in row order), their
    phase-start z and pending word proposals (M x n), the global c_k.
    Returns the row's new z and doc proposals, in row order."""
    n = len(z_pre)
    o = oracle.Oracle(np.asarray(word_ids_row, np.uint32), np.zeros(n, np.uint32), V, 1, K, M,
                      alpha, beta, seed=seed)
    o.init()
    o.set_csc_state(np.asarray(z_pre, np.int32), np.asarray(p_pre, np.int32))
    o.set_token_offsets(0, csr_off)
    o.set_phase_state(ck, oracle.PH_DOC, iteration)
    o.doc_phase()
    return o.csc()
