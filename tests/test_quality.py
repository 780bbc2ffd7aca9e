"""Quality studies on synthetic corpora, the analogues of Section 6.3: the
effect of the number of MH steps M, and delayed (per-phase) against instant
count updates.  These check the paper's qualitative claims on the oracle, not
parity: more MH steps per token converge faster per iteration, and the
delayed-update sampler converges at a rate close to that of a collapsed
Gibbs-MH sampler whose counts change as soon as a token moves (the instant-
update variant, which targets the collapsed posterior exactly).  The curves
are printed; the figures quoted in the design notes come from here."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.fixture(scope="module")
def corpus():
    return synth.WORKLOADS["tiny-lda-k16"].make()


def ll_curve(c, M, instant, iters, K=16, alpha=50.0 / 16, beta=0.01, seed=1):
    o = oracle.Oracle(c.word_ids, c.doc_ids, c.V, c.D, K, M, alpha, beta, seed=seed)
    o.init()
    out = [o.log_likelihood()]
    for _ in range(iters):
        if instant:
            o.instant_iterate(1)
        else:
            o.iterate(1)
        out.append(o.log_likelihood())
    return np.array(out)


def test_more_mh_steps_converge_faster(corpus):
    """Larger M: higher log likelihood at the same iteration (Section 6.3,
    effect of M)."""
    curves = {M: ll_curve(corpus, M, False, 20) for M in (1, 2, 4)}
    for M, cv in curves.items():
        print(f"M={M}: LL at iterations 1, 5, 10, 20: {cv[[1, 5, 10, 20]].round(0)}")
    for it in (5, 10, 20):
        assert curves[1][it] < curves[2][it] < curves[4][it], it


def test_delayed_updates_converge_close_to_instant_updates(corpus):
    """Delayed against instant count updates (Section 6.3): both chains climb
    from the same start, and after 50 iterations the delayed-update chain is
    behind the instant-update one by a small fraction of the likelihood it
    gained."""
    for M in (1, 2):
        d = ll_curve(corpus, M, False, 50)
        i = ll_curve(corpus, M, True, 50)
        print(f"M={M}: delayed {d[[1, 5, 10, 20, 50]].round(0)}, instant {i[[1, 5, 10, 20, 50]].round(0)}")
        assert d[0] == i[0]
        assert d[50] > d[10] > d[1] and i[50] > i[10] > i[1]
        gain = d[50] - d[0]
        assert abs(i[50] - d[50]) < 0.2 * gain, (d[50], i[50], gain)
