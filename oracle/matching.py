"""Exact diagram distances on tiny inputs (ground truth for the pins).

* ``dp_bruteforce``: the definition of d_p^p (section 2, eq. of d_p) by
  enumerating every partial matching between the two point sets.
* ``ot_assignment``: the exact optimal transport value L_C of Proposition 1,
  as the assignment problem built in its proof (repeat the diagonal row of C
  once per point of the first diagram and the diagonal column once per point
  of the second, zero block between the two diagonal copies).  Solved with
  ``scipy.optimize.linear_sum_assignment``, a library primitive.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.optimize import linear_sum_assignment


def _diag_cost(x, p):
    s, t = float(x[0]), float(x[1])
    mid = 0.5 * (s + t)                      # orthogonal projection onto the diagonal
    return abs(s - mid) ** p + abs(t - mid) ** p


def _pair_cost(x, y, p):
    return abs(float(x[0]) - float(y[0])) ** p + abs(float(x[1]) - float(y[1])) ** p


def dp_bruteforce(D1, D2, p: float = 2.0) -> float:
    """min over partial matchings of sum ||x - y||_p^p + sum_unmatched ||s - pi(s)||_p^p."""
    D1 = np.asarray(D1, np.float64).reshape(-1, 2)
    D2 = np.asarray(D2, np.float64).reshape(-1, 2)
    n1, n2 = len(D1), len(D2)
    best = math.inf
    for k in range(min(n1, n2) + 1):
        for left in itertools.combinations(range(n1), k):
            for right in itertools.permutations(range(n2), k):
                cost = 0.0
                for i, j in zip(left, right):
                    cost += _pair_cost(D1[i], D2[j], p)
                ml, mr = set(left), set(right)
                cost += sum(_diag_cost(D1[i], p) for i in range(n1) if i not in ml)
                cost += sum(_diag_cost(D2[j], p) for j in range(n2) if j not in mr)
                best = min(best, cost)
    return best


def hist_points(hist, d: int) -> np.ndarray:
    """Point list of a histogram: cell (i, j) at (i/d, j/d), repeated by its integer count."""
    hist = np.asarray(hist)
    pts = []
    for i in range(d):
        for j in range(d):
            c = int(round(hist[i, j]))
            pts.extend([(i / d, j / d)] * c)
    return np.asarray(pts, np.float64).reshape(-1, 2)


def ot_assignment(D1, D2, p: float = 2.0) -> float:
    """L_C(D1 + R D2, D2 + R D1) as an (n1 + n2) x (n1 + n2) assignment problem."""
    D1 = np.asarray(D1, np.float64).reshape(-1, 2)
    D2 = np.asarray(D2, np.float64).reshape(-1, 2)
    n1, n2 = len(D1), len(D2)
    n = n1 + n2
    if n == 0:
        return 0.0
    Ct = np.zeros((n, n))
    for i in range(n1):
        for j in range(n2):
            Ct[i, j] = _pair_cost(D1[i], D2[j], p)
        Ct[i, n2:] = _diag_cost(D1[i], p)          # D1 point -> one of n1 diagonal copies
    for j in range(n2):
        Ct[n1:, j] = _diag_cost(D2[j], p)          # one of n2 diagonal copies -> D2 point
    r, c = linear_sum_assignment(Ct)
    return float(Ct[r, c].sum())
