"""Launch-parameter tuner for the BF16 -> FP32 switch point.

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


def pick_fastest(times_ms: dict) -> float:
    """The key with the smallest median time (ties go to the larger switch
    point, which runs fewer FP32 iterations)."""
    if not times_ms:
        raise ValueError("no candidates")
    med = {k: float(np.median(v)) for k, v in times_ms.items()}
    return min(med, key=lambda k: (med[k], -k))


def tune_switch_tol(hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor, ib: torch.Tensor, d: int,
                    gamma: float, tol: float, max_iter: int = 5000, fractions=DEFAULT_FRACTIONS, reps: int = 3,
                    p: float = 2.0) -> dict:
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
                     device=hist_a.device.index) as ctx:
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
            times[sw] = ts
            it = out.iters.sum(dim=0).cpu().tolist()
            iters[sw] = (int(it[0]), int(it[1]))
    return {"switch_tol": pick_fastest(times), "ms": times, "iters": iters}
