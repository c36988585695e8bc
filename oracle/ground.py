"""Ground space of the diagram OT problem: discretisation, costs, kernels.

Readings of the paper taken here (each stated once):

* Grid units.  The 1-D cost is written |i - j|^p in index units in section 3
  ("Convolutions"); with the experiments' gamma in [5e-4, 1e-1] that only
  makes sense in [0,1] coordinates, so c_ij = (|i - j| h)^p with h = 1/d.
* Diagonal cost.  ||x - pi_Delta(x)||_p^p with the orthogonal projection onto
  the diagonal (section 2, eq. of d_p): for x = (s, t) this is
  2 (|t - s| / 2)^p.  On the grid the cell (i, j) is at (i h, j h), so
  c_Delta[i, j] = 2 (|j - i| h / 2)^p.
* Histogram orientation: row index = birth, column index = death.
* Discretisation (supplementary, "Error control due to discretization"): a
  point (b, t) goes to cell (floor(b d), floor(t d)), clipped to d - 1 so that
  the value 1.0 lands in the last cell.
"""
from __future__ import annotations

import numpy as np


def discretize(points, d: int) -> np.ndarray:
    """Histogram of a diagram on the d x d grid (float64 counts).

    Raises ``ValueError`` for points outside [0,1]^2 or with birth > death.
    The cell index is computed in float64 from the (float32) input, which is
    exact for any float32 value times an integer d < 2^24.
    """
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    h = np.zeros((d, d), dtype=np.float64)
    if pts.size == 0:
        return h
    if not np.all(np.isfinite(pts)):
        raise ValueError("non-finite point")
    if np.any(pts < 0.0) or np.any(pts > 1.0):
        raise ValueError("point outside [0,1]^2")
    if np.any(pts[:, 0] > pts[:, 1]):
        raise ValueError("birth > death")
    i = np.minimum(np.floor(pts[:, 0] * d).astype(np.int64), d - 1)
    j = np.minimum(np.floor(pts[:, 1] * d).astype(np.int64), d - 1)
    np.add.at(h, (i, j), 1.0)
    return h


def cost_1d(d: int, p: float = 2.0) -> np.ndarray:
    """c[i, k] = (|i - k| / d)^p  (section 3, "Convolutions", in [0,1] units)."""
    idx = np.arange(d, dtype=np.float64)
    return (np.abs(idx[:, None] - idx[None, :]) / d) ** p


def cost_diag(d: int, p: float = 2.0) -> np.ndarray:
    """c_Delta[i, j] = 2 (|j - i| / (2 d))^p: cost of sending cell (i, j) to the diagonal."""
    idx = np.arange(d, dtype=np.float64)
    return 2.0 * (np.abs(idx[None, :] - idx[:, None]) / (2.0 * d)) ** p


def kernel_1d(d: int, gamma: float, p: float = 2.0) -> np.ndarray:
    """k = exp(-c / gamma)."""
    return np.exp(-cost_1d(d, p) / gamma)


def kernel_diag(d: int, gamma: float, p: float = 2.0) -> np.ndarray:
    """k_Delta = exp(-c_Delta / gamma)."""
    return np.exp(-cost_diag(d, p) / gamma)


def dense_cost(d: int, p: float = 2.0) -> np.ndarray:
    """Dense (d^2+1) x (d^2+1) cost of section 3 ("Convolutions").

    Flat index of cell (i, j) is i*d + j; the diagonal bin is the last index.
    C[(i,j),(k,l)] = c[i,k] + c[j,l];  C[(i,j),Delta] = C[Delta,(i,j)] = c_Delta[i,j];
    C[Delta, Delta] = 0.
    """
    c = cost_1d(d, p)
    n = d * d
    C = np.zeros((n + 1, n + 1), dtype=np.float64)
    C[:n, :n] = (c[:, None, :, None] + c[None, :, None, :]).reshape(n, n)
    cd = cost_diag(d, p).reshape(n)
    C[:n, n] = cd
    C[n, :n] = cd
    return C


def marginals(hist_a: np.ndarray, hist_b: np.ndarray):
    """Marginals of Proposition 1 on the grid: a = (hist_a, |hist_b|), b = (hist_b, |hist_a|)."""
    a = np.append(np.asarray(hist_a, np.float64).ravel(), float(np.sum(hist_b)))
    b = np.append(np.asarray(hist_b, np.float64).ravel(), float(np.sum(hist_a)))
    return a, b
