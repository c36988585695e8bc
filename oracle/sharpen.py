"""Entropic sharpening of a barycenter, FP64 (test infrastructure only).

Section 4 (the paragraph after Algorithm 2) observes that the smoothed
barycenters come out smeared and points to entropic sharpening (section 6.1
of the convolutional-Wasserstein paper it cites) for more spiked diagrams,
leaving it to future work.  The paper gives no formula; readings taken here:

* Entropy of a histogram z >= 0 of mass M = sum z: the Shannon entropy
  H(z) = -sum_c p_c log p_c of p = z / M over the cells with z_c > 0.  The
  diagonal bin is not part of z (the operator R ties it to the mass).
* Sharpening to a target entropy h0: if H(z) <= h0, z is returned unchanged
  (beta = 1).  Otherwise z is replaced by M p^beta / sum_c p_c^beta with the
  beta > 1 at which that histogram's entropy is h0.  Along beta the entropy
  falls monotonically towards log n_max, n_max the number of cells at the
  maximum of z; when h0 <= log n_max that limit (the mass M spread evenly over
  the maximal cells, beta = inf) is returned.
* Mass, support and the order of the cells by mass are kept.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import xlogy


def entropy(z) -> float:
    """Shannon entropy of z / sum(z) over its positive cells (natural log)."""
    z = np.asarray(z, np.float64).ravel()
    z = z[z > 0]
    if z.size == 0:
        return 0.0
    p = z / z.sum()
    return float(-np.sum(xlogy(p, p)))     # 0 log 0 = 0 where a share underflows


def power_normalised(z, beta):
    """M p^beta / sum p^beta on the positive cells of z (0 elsewhere)."""
    z = np.asarray(z, np.float64)
    out = np.zeros_like(z)
    pos = z > 0
    if not np.any(pos):
        return out
    M = z[pos].sum()
    lz = np.log(z[pos]) - np.log(z[pos].max())     # <= 0: no overflow at large beta
    w = np.exp(beta * lz)
    out[pos] = M * w / w.sum()
    return out


def sharpen(z, h0: float):
    """Returns ``(z_sharp, beta)`` per the readings above."""
    z = np.asarray(z, np.float64)
    pos = z > 0
    if not np.any(pos) or entropy(z) <= h0:
        return z.copy(), 1.0
    zmax = z[pos].max()
    n_max = int(np.count_nonzero(z == zmax))
    if h0 <= math.log(n_max):
        out = np.where(z == zmax, z[pos].sum() / n_max, 0.0)
        return out, math.inf
    f = lambda b: entropy(power_normalised(z, b)) - h0
    hi = 2.0
    while f(hi) > 0:
        hi *= 2.0
    beta = brentq(f, 1.0, hi, xtol=1e-14, rtol=4 * np.finfo(float).eps, maxiter=500)
    return power_normalised(z, beta), float(beta)


def quantize(z) -> np.ndarray:
    """Quantisation of a barycenter to point counts (the paper's other pointer
    to spikier barycenters, with no formula; reading taken here): each cell's
    mass, in point units, rounded to the nearest integer, halves upwards
    (floor(z + 1/2), exact for float32 input).  The result is a histogram of
    integer counts, that is a persistence diagram on the grid."""
    z = np.asarray(z, np.float64)
    return np.floor(z + 0.5).astype(np.int64)
