"""k-means on persistence diagrams (section 5): assignment by Algorithm 1,
centroids by Algorithm 2.

Readings taken here: the distance of diagram n to centroid c is
S_C^gamma(a_n + R z_c, z_c + R a_n) (diagram first); ties go to the lowest
centroid index; initial centroids are k distinct diagrams chosen by a seeded
generator; a cluster that loses all its members keeps its centroid.
"""
from __future__ import annotations

import numpy as np

from . import barycenter as bary
from . import ground, sinkhorn


def assign(hists, centroids, gamma, p=2.0, tol=1e-3, max_iter=1000, C=None):
    """Return ``(labels int32 [N], dist float64 [N, k], iters int [N, k])``."""
    d = np.asarray(hists[0]).shape[0]
    if C is None:
        C = ground.dense_cost(d, p)
    N, k = len(hists), len(centroids)
    dist = np.zeros((N, k))
    iters = np.zeros((N, k), dtype=np.int64)
    for n in range(N):
        for c in range(k):
            a, b = ground.marginals(hists[n], centroids[c])
            r = sinkhorn.solve(a, b, C, gamma, tol=tol, max_iter=max_iter)
            dist[n, c] = r.cost
            iters[n, c] = r.iters
    labels = np.argmin(dist, axis=1).astype(np.int32)    # first minimum: lowest index
    return labels, dist, iters


def lloyd(hists, k, rounds, gamma, p=2.0, tol=1e-3, seed=0, lam=5.0, max_outer=10,
          energy_rtol=0.01, C=None):
    hists = [np.asarray(h, np.float64) for h in hists]
    d = hists[0].shape[0]
    if C is None:
        C = ground.dense_cost(d, p)
    rng = np.random.default_rng(seed)
    init = rng.choice(len(hists), size=k, replace=False)
    cents = [hists[i].copy() for i in init]
    history = []
    labels = None
    for _ in range(rounds):
        labels, dist, _ = assign(hists, cents, gamma, p, tol, C=C)
        history.append(float(dist[np.arange(len(hists)), labels].sum()))
        for c in range(k):
            members = [hists[i] for i in np.flatnonzero(labels == c)]
            if members:
                cents[c] = bary.barycenter(members, gamma, p, lam=lam, tol=tol,
                                           max_outer=max_outer, energy_rtol=energy_rtol, C=C).z
    return cents, labels, history
