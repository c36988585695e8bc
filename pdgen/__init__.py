"""Seeded synthetic persistence diagrams.

This module only draws random points: it holds none of the transport
arithmetic, so both the FP64 oracle and the GPU path may use it as their
common source of inputs.  Every generator takes a ``numpy.random.Generator``
(or a seed) and consumes it in the fixed order documented on the function, so
a given seed always yields the same diagrams.

A persistence diagram is an ``(n, 2)`` float32 array of (birth, death) pairs
with ``0 <= birth <= death <= 1`` (the paper assumes supports in
``[0, 1]^2`` above the diagonal, section 3, "Discretization").  Diagrams are
float32 because that is what the device boundary takes; every consumer reads
the same float32 values.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gen",
    "as_rng",
    "pair_single",
    "pairs_batch",
    "bary_set",
    "kmeans_set",
    "serve_stream",
    "to_csr",
]

#: Mean (scale) of the exponential persistence draw, death = birth + Exp.
PERSISTENCE_SCALE = 0.2


def as_rng(seed_or_rng) -> np.random.Generator:
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.default_rng(seed_or_rng)


def gen(rng: np.random.Generator, n: int) -> np.ndarray:
    """Random diagram with ``n`` points.

    Draw order: ``n`` births ``U[0,1)``, then ``n`` persistences
    ``Exp(scale=0.2)``; death = min(birth + persistence, 1).
    """
    b = rng.random(n)
    t = np.minimum(b + rng.exponential(PERSISTENCE_SCALE, n), 1.0)
    return np.stack([b, t], axis=1).astype(np.float32)


def _project(pts: np.ndarray) -> np.ndarray:
    """Clip to [0,1]^2 and lift death to at least birth (back above the diagonal)."""
    p = np.clip(pts, 0.0, 1.0)
    p[:, 1] = np.maximum(p[:, 1], p[:, 0])
    return p.astype(np.float32)


def pair_single(seed=0, n1: int = 20, n2: int = 30):
    """One pair: ``D1 = gen(n1)`` then ``D2 = gen(n2)`` from one generator."""
    rng = as_rng(seed)
    return gen(rng, n1), gen(rng, n2)


def pairs_batch(seed=0, n_pairs: int = 1024, lo: int = 50, hi: int = 500):
    """``n_pairs`` pairs with point counts ``U{lo..hi}``.

    Per pair, in order: ``(n1, n2) = rng.integers(lo, hi + 1, 2)``, then
    ``D1 = gen(n1)``, ``D2 = gen(n2)``.  Returns two lists of diagrams.
    """
    rng = as_rng(seed)
    d1, d2 = [], []
    for _ in range(n_pairs):
        n1, n2 = rng.integers(lo, hi + 1, 2)
        d1.append(gen(rng, int(n1)))
        d2.append(gen(rng, int(n2)))
    return d1, d2


def bary_set(seed=0, n_diag: int = 256, lo: int = 100, hi: int = 400,
             template_size: int = 400, sigma: float = 0.02, noise_frac: float = 0.1):
    """Perturbations of one template diagram.

    Order: template ``T = gen(template_size)``; then per diagram
    ``n = rng.integers(lo, hi + 1)``, ``k = round((1 - noise_frac) * n)``
    template points drawn with replacement, Gaussian jitter ``N(0, sigma^2)``
    per coordinate, then ``n - k`` fresh ``gen`` points; finally clip to
    [0,1]^2 and lift deaths to at least births.
    """
    rng = as_rng(seed)
    tmpl = gen(rng, template_size).astype(np.float64)
    out = []
    for _ in range(n_diag):
        n = int(rng.integers(lo, hi + 1))
        k = int(round((1.0 - noise_frac) * n))
        idx = rng.integers(0, template_size, k)
        pts = tmpl[idx] + rng.normal(0.0, sigma, (k, 2))
        extra = gen(rng, n - k).astype(np.float64)
        out.append(_project(np.concatenate([pts, extra], axis=0)))
    return out


def kmeans_set(seed=0, n_diag: int = 4000, n_templates: int = 10,
               template_size: int = 200, sigma: float = 0.03, change: float = 0.2):
    """Diagrams drawn around ``n_templates`` templates.

    Order: templates ``gen(template_size)`` each; per diagram ``i`` (template
    ``i mod n_templates``): jitter ``N(0, sigma^2)``, project, then
    ``r ~ U[-change, change]``: drop ``round(|r| * template_size)`` random
    points if ``r < 0``, else append ``round(r * template_size)`` ``gen``
    points.  Returns ``(diagrams, labels)``.
    """
    rng = as_rng(seed)
    tmpls = [gen(rng, template_size).astype(np.float64) for _ in range(n_templates)]
    out, labels = [], []
    for i in range(n_diag):
        c = i % n_templates
        pts = _project(tmpls[c] + rng.normal(0.0, sigma, tmpls[c].shape)).astype(np.float64)
        r = rng.uniform(-change, change)
        m = int(round(abs(r) * template_size))
        if r < 0:
            keep = rng.permutation(len(pts))[: max(len(pts) - m, 0)]
            pts = pts[np.sort(keep)]
        elif m > 0:
            pts = np.concatenate([pts, gen(rng, m).astype(np.float64)], axis=0)
        out.append(pts.astype(np.float32))
        labels.append(c)
    return out, np.asarray(labels, dtype=np.int32)


def serve_stream(seed=0, rate: float = 2000.0, duration: float = 1.0,
                 grids=(50, 100, 200), mu: float = 5.0, sigma: float = 0.7):
    """Poisson request stream for a serving loop.

    Per request, in order: inter-arrival ``Exp(1/rate)``, kind
    (``0`` = distance, ``1`` = assign) with probability 1/2, grid drawn
    uniformly from ``grids``, then one or two diagrams with
    ``max(1, round(lognormal(mu, sigma)))`` points each.  Returns a list of
    dicts with keys ``t``, ``kind``, ``d``, ``diagrams``.
    """
    rng = as_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        kind = int(rng.integers(0, 2))
        d = int(grids[int(rng.integers(0, len(grids)))])
        nd = 2 if kind == 0 else 1
        dg = [gen(rng, max(1, int(round(rng.lognormal(mu, sigma))))) for _ in range(nd)]
        reqs.append({"t": t, "kind": kind, "d": d, "diagrams": dg})
    return reqs


def to_csr(diagrams):
    """Concatenate diagrams: ``(pts float32 [total, 2], offsets int64 [n + 1])``."""
    counts = np.array([len(x) for x in diagrams], dtype=np.int64)
    offsets = np.zeros(len(diagrams) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    if len(diagrams):
        pts = np.concatenate([np.asarray(x, np.float32).reshape(-1, 2) for x in diagrams], axis=0)
    else:
        pts = np.zeros((0, 2), np.float32)
    return np.ascontiguousarray(pts, dtype=np.float32), offsets
