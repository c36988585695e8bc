"""Error control of section 3 ("Upper and Lower Bounds"), FP64, dense.

TEST INFRASTRUCTURE ONLY (see the package docstring).

After t Sinkhorn iterations with scalings (u_t, v_t) the paper brackets the
exact transport value L_C(a, b) between

* an upper bound M_t = <R_t, C>, where R_t is the rounding of the plan
  P_t = diag(u_t) K diag(v_t) onto the transport polytope Pi(a, b) by the
  rounding algorithm of Altschuler et al. recalled in the supplementary
  material (Proposition 4 gives a separable form of the same number), and
* a lower bound m_t = <alpha^{c cbar}, a> + <alpha^c, b>, where alpha = gamma
  log u_t and the c-transform / cbar-transform are the usual inf-convolutions
  with C (the dual variables they produce satisfy alpha_i + beta_j <= C_ij).

Both are computed here from their definitions on the dense (d^2+1)-point
ground space: the dense plan, the dense rounding, the dense transforms.

Readings taken here:

* Sign of the c-transform.  The transform is printed with a max over
  C_ij - alpha_i; only the infimum gives feasible dual variables, so that a
  lower bound follows from weak duality.  The oracle takes the min.
* Domain of the transforms.  Both transforms run over every point of the
  ground space (all d^2 grid cells, those below the diagonal included, and
  the diagonal bin), as on the paper's Eulerian grid; alpha = -inf where
  u_t = 0 (off supp(a)), so those points never attain the min.
* Rows of P with r(P)_i = 0 keep the factor 1 in the first rounding step
  (min(r_i / 0, 1) = 1); the row is zero either way.  The same for columns.
* The rank-one correction divides by ||e_c||_1 (with the diagonal bin); when
  it is 0 the rounded plan is P'' itself.
"""
from __future__ import annotations

import math

import numpy as np


def round_to_feasible(P, r, c):
    """F(P) in Pi(r, c): row scaling down to r, column scaling down to c, then
    the rank-one correction e_r e_c^T / ||e_c||_1 (rounding algorithm of the
    supplementary material, after Altschuler et al.)."""
    P = np.asarray(P, np.float64)
    r = np.asarray(r, np.float64)
    c = np.asarray(c, np.float64)
    rp = P.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        X = np.where(rp > 0, np.minimum(r / rp, 1.0), 1.0)
    P1 = X[:, None] * P
    cp = P1.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        Y = np.where(cp > 0, np.minimum(c / cp, 1.0), 1.0)
    P2 = P1 * Y[None, :]
    er = r - P2.sum(axis=1)
    ec = c - P2.sum(axis=0)
    n1 = np.abs(ec).sum()
    if n1 == 0.0:
        return P2
    return P2 + np.outer(er, ec) / n1


def dense_plan(log_u, log_v, C, gamma):
    """P_t = diag(u) K diag(v) with K = exp(-C / gamma), from the log scalings
    (-inf where a scaling vanishes)."""
    with np.errstate(invalid="ignore"):
        E = np.asarray(log_u)[:, None] + np.asarray(log_v)[None, :] - np.asarray(C) / gamma
    E = np.where(np.isfinite(E), E, -np.inf)
    return np.exp(E)


def upper_bound(log_u, log_v, a, b, C, gamma) -> float:
    """M_t = <F(P_t), C> with F the rounding onto Pi(a, b)."""
    F = round_to_feasible(dense_plan(log_u, log_v, C, gamma), a, b)
    return math.fsum((F * C).sum(axis=1).tolist())


def c_transform(alpha, C):
    """alpha^c_j = min_i (C_ij - alpha_i)."""
    alpha = np.asarray(alpha, np.float64)
    return np.min(np.asarray(C) - alpha[:, None], axis=0)


def cbar_transform(beta, C):
    """beta^cbar_i = min_j (C_ij - beta_j)."""
    beta = np.asarray(beta, np.float64)
    return np.min(np.asarray(C) - beta[None, :], axis=1)


def dual_bound(alpha, a, b, C) -> float:
    """<alpha^{c cbar}, a> + <alpha^c, b>: the dual objective of the feasible
    pair (alpha^{c cbar}, alpha^c), a lower bound of L_C(a, b)."""
    ac = c_transform(alpha, C)
    acc = cbar_transform(ac, C)
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    sa, sb = a > 0, b > 0
    return math.fsum((a[sa] * acc[sa]).tolist()) + math.fsum((b[sb] * ac[sb]).tolist())


def lower_bound(log_u, a, b, C, gamma) -> float:
    """m_t for alpha = gamma log u_t."""
    return dual_bound(gamma * np.asarray(log_u, np.float64), a, b, C)
