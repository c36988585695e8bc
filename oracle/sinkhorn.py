"""Algorithm 1 of the paper on the dense (d^2+1)-point ground space, in FP64.

The method's output is the Sinkhorn iterate at stopping, not an exact
optimum: after t iterations of the Sinkhorn map (section 2, eq. of the map S)
the plan is P_t = diag(u_t) K diag(v_t) and the returned value is the Sinkhorn
divergence <P_t, C> (section 2; Algorithm 1 returns it for every pair).

Readings taken here:

* Update order.  The map S is written as a simultaneous update; the oracle
  runs the usual alternating form: u from v, then v from the new u.  One
  iteration is both half steps.  Both forms have the same fixed point.
* Initialisation.  Algorithm 1 takes an initial (u, v); the default is v = 1
  on all d^2 + 1 entries and the first half step updates u.
* Empty bins.  u = 0 where a = 0 and v = 0 where b = 0.
* Stopping.  dist(P, Pi(a,b)) = ||P 1 - a||_1 + ||P^T 1 - b||_1 (section 3,
  after the error bound), divided by the common mass m of a and b, checked
  after every iteration; the loop also stops at ``max_iter``.
* Stabilisation (the paper is silent).  The scaling vectors are kept as
  u = exp(alpha) * u~, v = exp(beta) * v~ with the kernel
  K~ = exp(alpha (+) beta - C / gamma); whenever u~ or v~ leaves
  [1e-50, 1e50] on its support, log u~ and log v~ are moved into alpha and
  beta.  In exact arithmetic the iterates are unchanged; in FP64 it keeps
  every scaling and every plan entry representable.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import logsumexp

from . import ground

_BOUND = 1e50


class OracleRangeError(ArithmeticError):
    """A kernel product vanished on the support: the iterate is not representable."""


@dataclass
class SinkhornResult:
    cost: float                 # <P_t, C>
    iters: int                  # t, number of full (u, v) iterations run
    err: float                  # dist(P_t, Pi(a, b)) / m
    log_u: np.ndarray           # natural log of u_t (length d^2+1, -inf where a == 0)
    log_v: np.ndarray           # natural log of v_t
    absorptions: int = 0
    errs: list = field(default_factory=list)
    mass: float = 0.0


def _gibbs(alpha, beta, C, gamma):
    E = C * (-1.0 / gamma)
    E += alpha[:, None]
    E += beta[None, :]
    np.exp(E, out=E)
    return E


def _scale(target, denom):
    out = np.zeros_like(target)
    s = target > 0
    bad = s & ~(np.isfinite(denom) & (denom > 0))
    if np.any(bad):
        raise OracleRangeError("K v vanished or overflowed on the support")
    out[s] = target[s] / denom[s]
    return out


def plan_cost(ut, vt, Kt, C, rows=2048) -> float:
    """<diag(u) K~ diag(v), C> summed row block by row block, outer sum with fsum."""
    parts = []
    n = C.shape[0]
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        rv = (Kt[r0:r1] * C[r0:r1]) @ vt
        parts.extend((ut[r0:r1] * rv).tolist())
    return math.fsum(parts)


def solve(a, b, C, gamma, tol=0.0, max_iter=1000, log_v0=None, record=False) -> SinkhornResult:
    """Alternating Sinkhorn on marginals ``a``, ``b`` (same total mass) and cost ``C``.

    ``log_v0`` (natural log of the initial v, -inf allowed) is the warm start;
    ``None`` means v = 1 everywhere.
    """
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = a.shape[0]
    sa, sb = a > 0, b > 0
    m = float(a.sum())
    alpha = np.zeros(n)
    if log_v0 is None:
        beta = np.zeros(n)
        vt = np.ones(n)
    else:
        lv = np.asarray(log_v0, np.float64)
        fin = np.isfinite(lv)
        beta = np.where(fin, lv, -np.inf)
        vt = fin.astype(np.float64)
    Kt = _gibbs(alpha, beta, C, gamma)
    Kv = Kt @ vt
    absorptions = 0
    errs = []
    t = 0
    err = math.inf
    ut = np.zeros(n)
    if m <= 0.0:
        return SinkhornResult(0.0, 0, 0.0, np.full(n, -np.inf), np.full(n, -np.inf), 0, [], 0.0)
    for t in range(1, max_iter + 1):
        ut = _scale(a, Kv)
        Ktu = Kt.T @ ut
        vt = _scale(b, Ktu)
        Kv = Kt @ vt
        err = (np.abs(ut * Kv - a).sum() + np.abs(vt * Ktu - b).sum()) / m
        if record:
            errs.append(err)
        if err <= tol or t == max_iter:
            break
        us, vs = ut[sa], vt[sb]
        if (us.max() > _BOUND or us.min() < 1.0 / _BOUND
                or vs.max() > _BOUND or vs.min() < 1.0 / _BOUND):
            with np.errstate(divide="ignore"):
                alpha = np.where(sa, alpha + np.log(ut), -np.inf)
                beta = np.where(sb, beta + np.log(vt), -np.inf)
            ut = sa.astype(np.float64)
            vt = sb.astype(np.float64)
            Kt = _gibbs(alpha, beta, C, gamma)
            Kv = Kt @ vt
            absorptions += 1
    cost = plan_cost(ut, vt, Kt, C)
    with np.errstate(divide="ignore"):
        log_u = np.where(sa, alpha + np.log(np.where(sa, ut, 1.0)), -np.inf)
        log_v = np.where(sb, beta + np.log(np.where(sb, vt, 1.0)), -np.inf)
    return SinkhornResult(cost, t, float(err), log_u, log_v, absorptions, errs, m)


def sinkhorn(hist_a, hist_b, gamma, p=2.0, tol=0.0, max_iter=1000, log_v0=None, C=None,
             record=False) -> SinkhornResult:
    """Algorithm 1 for one pair of d x d histograms: marginals of Proposition 1."""
    hist_a = np.asarray(hist_a, np.float64)
    d = hist_a.shape[0]
    if C is None:
        C = ground.dense_cost(d, p)
    a, b = ground.marginals(hist_a, hist_b)
    return solve(a, b, C, gamma, tol=tol, max_iter=max_iter, log_v0=log_v0, record=record)


def plan(res: SinkhornResult, C, gamma) -> np.ndarray:
    """Dense P_t = diag(u) K diag(v), from the log scalings (small sizes only)."""
    E = res.log_u[:, None] + res.log_v[None, :] - C / gamma
    return np.exp(E)


def entropic_objective(P, C, gamma) -> float:
    """<P, C> - gamma h(P) with h(P) = -sum P (log P - 1) (section 2, entropic problem)."""
    pos = P > 0
    ent = np.sum(P[pos] * (np.log(P[pos]) - 1.0))
    return float(np.sum(P * C) + gamma * ent)


def solve_log(a, b, C, gamma, tol=0.0, max_iter=1000):
    """Same alternating iterations written with log-sum-exp (dense, small sizes only).

    Returns ``(cost, iters, err, log_u, log_v)``.  This is a second, independent
    formulation used to pin the stabilised scaling form above.
    """
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    sa, sb = a > 0, b > 0
    m = a.sum()
    G = -C / gamma
    lv = np.zeros(len(b))
    with np.errstate(divide="ignore"):
        la, lb = np.log(a), np.log(b)
    t, err = 0, math.inf
    lu = np.full(len(a), -np.inf)
    for t in range(1, max_iter + 1):
        lu = np.where(sa, la - logsumexp(G + lv[None, :], axis=1), -np.inf)
        lKtu = logsumexp(G + lu[:, None], axis=0)
        lv = np.where(sb, lb - lKtu, -np.inf)
        P = np.exp(G + lu[:, None] + lv[None, :])
        err = (np.abs(P.sum(1) - a).sum() + np.abs(P.sum(0) - b).sum()) / m
        if err <= tol or t == max_iter:
            break
    P = np.exp(G + lu[:, None] + lv[None, :])
    return math.fsum((P * C).ravel().tolist()), t, float(err), lu, lv
