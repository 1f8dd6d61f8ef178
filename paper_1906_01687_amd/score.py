"""Factor-match score of App. E: how close a fitted CP model is to a known one.

Columns of each factor matrix are normalised; the similarity of component j
of the reference with component j' of the estimate is the product over modes
of their column cosines; the score is the mean of these similarities under
the best one-to-one matching of components (the assignment problem, solved
exactly).  A score of at least 0.9 counts as recovery in the paper's
experiments (Sec. 5).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def factor_match_score(A_ref: Sequence[np.ndarray], A_est: Sequence[np.ndarray]) -> float:
    from scipy.optimize import linear_sum_assignment

    if len(A_ref) != len(A_est):
        raise ValueError("the two models have different numbers of modes")
    r = np.asarray(A_ref[0]).shape[1]
    sim = np.ones((r, np.asarray(A_est[0]).shape[1]))
    for a, b in zip(A_ref, A_est):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        na = np.linalg.norm(a, axis=0)
        nb = np.linalg.norm(b, axis=0)
        sim *= (a / np.where(na > 0, na, 1.0)).T @ (b / np.where(nb > 0, nb, 1.0))
    rows, cols = linear_sum_assignment(-sim)
    return float(sim[rows, cols].sum() / r)
