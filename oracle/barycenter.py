"""Algorithm 2 of the paper: smoothed barycenter of persistence diagrams.

The energy of a candidate x (a d x d histogram) is
E(x) = (1/N) sum_i S_C^gamma(x + R a_i, a_i + R x) (Algorithm 2, energy step).
Its smoothed gradient is given by Proposition 5,
grad = gamma (sum_i log u_i + R^T log v_i), and R^T log v_i is the constant
matrix (log v_i)_Delta, since R maps a histogram to its mass on the diagonal
bin.  x is updated multiplicatively, x <- x * exp(-lambda grad).

Readings taken here:

* The gradient is averaged over the N diagrams (the energy of Algorithm 2 is
  an average), so lambda does not scale with N.
* Initialisation: x uniform on the cells with j >= i (on and above the
  diagonal), total mass = the mean mass of the input diagrams.  The update is
  multiplicative, so x keeps that support.
* Inner Sinkhorn loops stop at the marginal-error tolerance and are warm
  started from the previous outer step's v_i.
* Outer loop: at step t the inner loops run for x_t and give E_t; the loop
  stops when |E_t / E_{t-1} - 1| < energy_rtol (section 5) or after
  ``max_outer`` steps and returns (x_t, E_t); otherwise x_{t+1} is the
  multiplicative update of x_t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import ground, sinkhorn


@dataclass
class BarycenterResult:
    z: np.ndarray           # d x d
    energy: float
    outer: int
    energies: list
    inner_iters: list


def uniform_init(d: int, mass: float) -> np.ndarray:
    z = np.triu(np.ones((d, d)))
    return z * (mass / z.sum())


def barycenter(hists, gamma, p=2.0, lam=5.0, tol=1e-3, max_inner=1000, max_outer=50,
               energy_rtol=0.01, z0=None, C=None) -> BarycenterResult:
    hists = [np.asarray(h, np.float64) for h in hists]
    d = hists[0].shape[0]
    n_cells = d * d
    if C is None:
        C = ground.dense_cost(d, p)
    N = len(hists)
    z = uniform_init(d, float(np.mean([h.sum() for h in hists]))) if z0 is None else np.array(z0, np.float64)
    warm = [None] * N
    energies, inner = [], []
    E_prev = None
    t = 0
    for t in range(max_outer):
        grad = np.zeros(n_cells)
        costs = []
        its = []
        for i, h in enumerate(hists):
            a, b = ground.marginals(z, h)
            res = sinkhorn.solve(a, b, C, gamma, tol=tol, max_iter=max_inner, log_v0=warm[i])
            warm[i] = res.log_v
            lu = res.log_u[:n_cells]
            grad += np.where(np.isfinite(lu), lu, 0.0) + res.log_v[n_cells]
            costs.append(res.cost)
            its.append(res.iters)
        E = float(np.mean(costs))
        energies.append(E)
        inner.append(its)
        if E_prev is not None and abs(E / E_prev - 1.0) < energy_rtol:
            break
        if t == max_outer - 1:
            break
        grad *= gamma / N
        z = np.where(z > 0, z * np.exp(-lam * grad.reshape(d, d)), 0.0)
        E_prev = E
    return BarycenterResult(z, energies[-1], t + 1, energies, inner)
