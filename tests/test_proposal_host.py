"""Host-side logic of the proposal training and evaluation loop (no GPU): threshold choice,
recall and agreement."""
import numpy as np

import paper_1403_2136_amd as mx
from paper_1403_2136_amd import proposal as P


def _labels(frags):
    a = np.zeros(len(frags), dtype=mx.TOP2_DTYPE)
    a["frag"][:, 0] = frags
    return a


def test_recall():
    cand = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 9]])
    assert P.recall(cand, _labels([2, 9, 9])).tolist() == [True, False, True]


def test_choose_margin_falls_back_the_smallest_margins():
    # reads 0..9 with margins 0.1..1.0; the misses are the reads with margins 0.1 and 0.3
    margins = np.arange(1, 11) / 10.0
    cand = np.zeros((10, 2), dtype=np.int64)
    labels = _labels(np.zeros(10, dtype=np.int64))
    cand[[0, 2], :] = 5                                  # label 0 missing for reads 0 and 2
    m32 = margins.astype(np.float32)
    tau = P.choose_margin(cand, m32, labels, 1.0)
    assert (m32 < tau).sum() == 3                      # reads with margins 0.1, 0.2, 0.3
    assert (m32 < P.choose_margin(cand, m32, labels, 0.8)).sum() == 0   # 8/10 already agree
    assert (m32 < P.choose_margin(np.zeros((10, 2), np.int64), m32, labels, 1.0)).sum() == 0


def test_agreements():
    a = np.zeros(3, dtype=mx.TOP2_DTYPE)
    b = np.zeros(3, dtype=mx.TOP2_DTYPE)
    a["frag"][:, 0] = [1, 2, 3]
    b["frag"][:, 0] = [1, 2, 4]
    a["score"][:, 0] = [5, 5, 5]
    b["score"][:, 0] = [5, 5, 5]
    assert abs(P.top1_agreement(a, b) - 2 / 3) < 1e-12
    assert P.score_agreement(a, b) == 1.0
