"""Write ``sinkhorn_golden.json``: FP64 oracle results that the GPU tests compare with.

Every value here comes from ``oracle/`` (dense (d^2+1)-point Sinkhorn of
Algorithm 1, FP64) on inputs drawn by ``pdgen``; nothing is taken from the
GPU path.  Two kinds of record:

* ``stop_1e-3``: the iteration count and cost at which the oracle first meets
  the marginal-error rule at tol = 1e-3 (pairs 0, 1, 2 of the batched-distance
  workload: 1024 pairs of 50..500 points, d = 100, gamma = 1e-3).
* ``converged``: the oracle run to err <= 1e-7 (or its iteration cap): the
  unique entropic fixed point that the BF16-with-refinement path is compared
  with at 1e-3 relative cost.  Pairs of the same workload whose diagrams are
  both large (they converge in about a thousand iterations), one pair of a
  dense upper-triangular histogram (the shape of a barycenter) against a
  diagram, and two pairs on a 136 x 136 grid (gamma = 2e-3).

Run from the repository root: ``python tests/golden/make_sinkhorn_golden.py``
(several minutes; one process per case).
"""
from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sinkhorn_golden.json")

CONV_TOL, CONV_MAX = 1e-7, 4000


def dense_centroid(d: int, mass: float):
    import numpy as np
    z = np.triu(np.ones((d, d)))
    return z * (mass / z.sum())


def inputs(case: dict):
    """The two histograms of a case, rebuilt from its generator description."""
    import numpy as np
    import pdgen
    from oracle import ground
    d = case["d"]
    g = case["gen"]
    if g["kind"] == "pairs_batch":
        d1, d2 = pdgen.pairs_batch(g["seed"], g["n_pairs"], g["lo"], g["hi"])
        q = case["index"]
        return ground.discretize(d1[q], d), ground.discretize(d2[q], d)
    if g["kind"] == "dense_vs_diagram":
        d1, _ = pdgen.pairs_batch(g["seed"], g["n_pairs"], g["lo"], g["hi"])
        h = ground.discretize(d1[case["index"]], d)
        # the dense histogram holds float32-representable values: the GPU reads it as float32
        z = dense_centroid(d, float(h.sum())).astype(np.float32).astype(np.float64)
        return (z, h) if g["dense_first"] else (h, z)
    raise ValueError(g["kind"])


def run(case: dict) -> dict:
    sys.path.insert(0, ROOT)
    from oracle import sinkhorn
    ha, hb = inputs(case)
    r = sinkhorn.sinkhorn(ha, hb, case["gamma"], p=2.0, tol=case["tol"], max_iter=case["max_iter"])
    out = dict(case)
    out.update({"cost": r.cost, "iters": int(r.iters), "err": float(r.err)})
    print(json.dumps({k: out[k] for k in ("name", "iters", "err", "cost")}), flush=True)
    return out


def cases():
    c2 = {"kind": "pairs_batch", "seed": 0, "n_pairs": 1024, "lo": 50, "hi": 500}
    out = []
    for q in (0, 1, 2):
        out.append({"name": f"c2_pair{q}_stop1e-3", "kind": "stop_1e-3", "gen": c2, "index": q, "d": 100,
                    "gamma": 1e-3, "tol": 1e-3, "max_iter": 5000})
    for q in (3, 17, 10, 0):
        out.append({"name": f"c2_pair{q}_converged", "kind": "converged", "gen": c2, "index": q, "d": 100,
                    "gamma": 1e-3, "tol": CONV_TOL, "max_iter": CONV_MAX})
    dense = {"kind": "dense_vs_diagram", "seed": 4, "n_pairs": 3, "lo": 50, "hi": 300, "dense_first": True}
    out.append({"name": "d100_dense_vs_diagram_converged", "kind": "converged", "gen": dense, "index": 0,
                "d": 100, "gamma": 1e-3, "tol": CONV_TOL, "max_iter": CONV_MAX})
    g136 = {"kind": "pairs_batch", "seed": 17, "n_pairs": 2, "lo": 60, "hi": 200}
    for q in (0, 1):
        out.append({"name": f"d136_pair{q}_converged", "kind": "converged", "gen": g136, "index": q, "d": 136,
                    "gamma": 2e-3, "tol": CONV_TOL, "max_iter": CONV_MAX})
    return out


def main():
    os.environ.setdefault("OMP_NUM_THREADS", "2")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "2")
    todo = cases()
    with ProcessPoolExecutor(max_workers=int(os.environ.get("GOLDEN_WORKERS", "4"))) as ex:
        res = list(ex.map(run, todo))
    rec = {"source": "oracle.sinkhorn.sinkhorn (dense FP64 Algorithm 1), inputs from pdgen; "
                     "written by tests/golden/make_sinkhorn_golden.py",
           "cases": res}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
