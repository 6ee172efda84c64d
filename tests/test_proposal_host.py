"""Host-side choice of the proposal's acceptance thresholds
(maxss_choose_acceptance, no GPU): against a brute force over every
threshold pair on random held-out sets, and on hand-made cases."""
import numpy as np
import pytest

import paper_1403_2136_amd as mx


def _agreement(margin, score, correct, tau, ms):
    acc = (margin >= tau) | ((ms >= 0) & (score >= ms))
    return 1.0 - (acc & (correct == 0)).sum() / margin.size, acc.mean()


def _brute(margin, score, correct, target):
    """The smallest min_score (or none) keeping the agreement >= target with
    the score rule alone, then the smallest margin of a read that rule
    leaves (or +inf) that keeps it."""
    n = margin.size
    ok = lambda a: a >= target - 1e-9
    ms = -1
    for s in sorted(set(score[score >= 0].tolist())):
        if ok(_agreement(margin, score, correct, np.inf, s)[0]):
            ms = s
            break
    tau = np.inf
    left = margin[(ms < 0) | (score < ms)]
    for t in sorted(set(left.tolist())):
        if ok(_agreement(margin, score, correct, t, ms)[0]):
            tau = t
            break
    return tau, ms


@pytest.mark.parametrize("seed", range(12))
def test_acceptance_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    score = rng.integers(-1, 12, n).astype(np.int32)
    margin = np.round(rng.uniform(0, 1, n), 1).astype(np.float32)   # ties
    correct = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    correct[score >= 9] = 1
    target = float(rng.choice([0.5, 0.8, 0.9, 0.95, 1.0]))
    tau, ms, acc, agr = mx.maxss_choose_acceptance(margin, score, correct, target)
    bt, bms = _brute(margin.astype(np.float64), score, correct, target)
    assert ms == bms
    assert tau == bt or (np.isinf(tau) and np.isinf(bt))
    a, f = _agreement(margin, score, correct, tau, ms)
    assert a >= target - 1e-6 and abs(a - agr) < 1e-6 and abs(f - acc) < 1e-6


def test_acceptance_hand_cases():
    # every best candidate right: everything is accepted by the lowest score
    tau, ms, acc, agr = mx.maxss_choose_acceptance([0.1, 0.2], [3, 5], [1, 1], 1.0)
    assert ms == 3 and acc == 1.0 and agr == 1.0
    # the best-scoring read is wrong: no score threshold keeps 100%; the
    # margin rule then accepts the right reads above the wrong one's margin
    tau, ms, acc, agr = mx.maxss_choose_acceptance([0.5, 0.9, 0.1], [9, 5, 4], [0, 1, 1], 1.0)
    assert ms == -1 and tau == np.float32(0.9) and abs(acc - 1 / 3) < 1e-6 and agr == 1.0
    # an empty held-out set accepts nothing
    tau, ms, acc, agr = mx.maxss_choose_acceptance([], [], [], 0.99)
    assert ms == -1 and np.isinf(tau) and acc == 0.0 and agr == 1.0
    with pytest.raises(mx.MaxssError):
        mx.maxss_choose_acceptance([0.1], [1], [1], 1.5)
