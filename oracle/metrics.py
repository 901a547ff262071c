"""Ranking metrics -- TEST INFRASTRUCTURE."""
import numpy as np


def auc(scores, labels) -> float:
    """Area under the ROC curve by the Mann-Whitney statistic, ties counted 1/2."""
    s = np.asarray(scores, dtype=np.float64)
    y = np.asarray(labels).astype(bool)
    pos, neg = s[y], s[~y]
    if pos.size == 0 or neg.size == 0:
        return float("nan")
    order = np.argsort(s, kind="mergesort")
    ranks = np.empty(s.size)
    sv = s[order]
    i = 0
    while i < s.size:                      # average ranks over ties
        j = i
        while j + 1 < s.size and sv[j + 1] == sv[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return float((ranks[y].sum() - pos.size * (pos.size + 1) / 2.0) / (pos.size * neg.size))
