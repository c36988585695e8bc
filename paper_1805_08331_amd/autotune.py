"""Launch-parameter tuners: the distance kernel's tiling, and the BF16 -> FP32
switch point.

Tiling (``tune_kernel``).  Two kernels compute the same Algorithm 1 solve
with different tiles and padding: the general kernel contracts over d padded
to 32, 64, 128 or 256 with 32 x 32 MFMA tiles over that grid; the resident
kernel (grids 33 to 100) contracts over d rounded up to the MFMA depth 16
(3 to 7 steps) and keeps the scaled kernels of both half steps in LDS between
refits.  Which is faster depends on d (how much padding each wastes) and on
how often the scales move, so the tuner times both on the caller's pairs and
caches the choice per (d, precision) for the process (``choose_kernel``).

With ``precision="bf16"`` a pair iterates with BF16 contractions until its
marginal error falls below ``switch_tol``, then with FP32 contractions until
it falls below ``tol``.  Every switch point gives a result that meets ``tol``
(the FP32 iterations decide the stopping point), so only the time changes:
switching late saves FP32 iterations; switching early avoids BF16 iterations
that stall near the BF16 rounding floor.  The best point depends on d, gamma,
tol and the diagrams, so ``tune_switch_tol`` times the caller's own pairs at
each candidate and returns the fastest.

Timing: one warm-up launch per candidate, then ``reps`` launches bracketed by
HIP events on the current stream (the library launches on that stream); the
median counts.  Candidates are fractions of ``tol``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Context, _lib, sinkhorn_dist_batch

DEFAULT_FRACTIONS = (0.5, 0.65, 0.8, 1.0)
KERNELS = ("resident", "general")
RESIDENT_GRIDS = range(33, 101)

_kernel_cache: dict = {}


def pick_fastest(times_ms: dict) -> float:
    """The key with the smallest median time (ties go to the larger switch
    point, which runs fewer FP32 iterations)."""
    if not times_ms:
        raise ValueError("no candidates")
    med = {k: float(np.median(v)) for k, v in times_ms.items()}
    return min(med, key=lambda k: (med[k], -k))


def tune_switch_tol(hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor, ib: torch.Tensor, d: int,
                    gamma: float, tol: float, max_iter: int = 5000, fractions=DEFAULT_FRACTIONS, reps: int = 3,
                    p: float = 2.0, kernel="auto") -> dict:
    """Time ``sinkhorn_dist_batch`` on pairs (hist_a[ia[q]], hist_b[ib[q]]) at
    ``switch_tol = f * tol`` for each f in ``fractions``.  Returns
    ``{"switch_tol": best, "ms": {switch_tol: [times]}, "iters": {switch_tol:
    (bf16, fp32) iteration totals}}``."""
    if reps < 1 or not fractions or any(f <= 0 for f in fractions):
        raise ValueError("reps >= 1 and positive fractions are required")
    times, iters = {}, {}
    for f in fractions:
        sw = float(f) * tol
        with Context(d, gamma, p=p, tol=tol, max_iter=max_iter, precision="bf16", switch_tol=sw,
                     device=hist_a.device.index, kernel=kernel) as ctx:
            ts, out = _time_batch(ctx, hist_a, hist_b, ia, ib, reps)
            times[sw] = ts
            it = out.iters.sum(dim=0).cpu().tolist()
            iters[sw] = (int(it[0]), int(it[1]))
    return {"switch_tol": pick_fastest(times), "ms": times, "iters": iters}


def _time_batch(ctx, hist_a, hist_b, ia, ib, reps):
    ws = ctx.workspace(_lib.PDSINK_OP_DIST, ia.numel())
    out = sinkhorn_dist_batch(ctx, hist_a, hist_b, ia, ib, ws=ws)      # warm-up, checks the indices
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sinkhorn_dist_batch(ctx, hist_a, hist_b, ia, ib, out=out, ws=ws, check_indices=False)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return ts, out


def tune_kernel(hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor, ib: torch.Tensor, d: int,
                gamma: float, tol: float, precision: str = "bf16", switch_tol: float = 1.5e-3,
                max_iter: int = 5000, reps: int = 3, p: float = 2.0) -> dict:
    """Time ``sinkhorn_dist_batch`` on the caller's pairs with each distance
    kernel ("resident", "general"; only "general" outside d in 33..100) and
    cache the fastest for (d, precision).  Returns ``{"kernel": best, "ms":
    {kernel: [times]}, "cost_rel": max relative cost difference between the
    kernels}``: both solve the same iteration, so their costs agree to the
    rounding of their contractions."""
    if reps < 1:
        raise ValueError("reps >= 1 is required")
    cands = KERNELS if d in RESIDENT_GRIDS else ("general",)
    times, costs = {}, {}
    for k in cands:
        with Context(d, gamma, p=p, tol=tol, max_iter=max_iter, precision=precision, switch_tol=switch_tol,
                     device=hist_a.device.index, kernel=k) as ctx:
            ts, out = _time_batch(ctx, hist_a, hist_b, ia, ib, reps)
            times[k] = ts
            costs[k] = out.cost.cpu().numpy()
    med = {k: float(np.median(v)) for k, v in times.items()}
    best = min(med, key=lambda k: (med[k], KERNELS.index(k)))
    rel = 0.0
    if len(costs) == 2:
        a, b = costs["resident"], costs["general"]
        rel = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))) if a.size else 0.0
    _kernel_cache[(int(d), str(precision))] = best
    return {"kernel": best, "ms": times, "median_ms": med, "cost_rel": rel}


def choose_kernel(d: int, precision: str = "bf16") -> str:
    """The kernel ``tune_kernel`` picked for (d, precision) in this process,
    else "auto" (the library's default for the grid)."""
    return _kernel_cache.get((int(d), str(precision)), "auto")
