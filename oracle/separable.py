"""Propositions 2 and 3 of the paper, written out in FP64.

These are the separable forms of the K application and of the transport cost
on the d x d grid plus the diagonal bin.  The oracle's Sinkhorn runs on the
dense kernel; these functions exist so that tests can check the dense path
against the paper's identities (and vice versa).
"""
from __future__ import annotations

import numpy as np

from . import ground


def tables(d: int, gamma: float, p: float = 2.0):
    """k, m = k * c, k_Delta, m_Delta = k_Delta * c_Delta (section 3, before Prop. 3)."""
    c = ground.cost_1d(d, p)
    cd = ground.cost_diag(d, p)
    k = np.exp(-c / gamma)
    kd = np.exp(-cd / gamma)
    return k, k * c, kd, kd * cd


def apply_K(U, u_delta, k, k_delta):
    """Proposition 2: K (U, u_Delta) = (k (k U^T)^T + u_Delta k_Delta, <U, k_Delta> + u_Delta)."""
    W = k @ (k @ U.T).T + u_delta * k_delta
    return W, float(np.sum(U * k_delta) + u_delta)


def transport_cost(U, u_delta, V, v_delta, k, m, m_delta):
    """Proposition 3: <diag(u) K diag(v), C> =
    ||U * (m (k V^T)^T + k (m V^T)^T)||_1 + u_Delta <V, m_Delta> + v_Delta <U, m_Delta>.

    (The supplementary proof spells the first term as the sum over cells of
    U times that matrix; both readings agree because every factor is >= 0.)
    """
    first = np.sum(U * (m @ (k @ V.T).T + k @ (m @ V.T).T))
    return float(first + u_delta * np.sum(V * m_delta) + v_delta * np.sum(U * m_delta))
