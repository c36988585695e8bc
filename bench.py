"""Benchmark: batched PD-pair Sinkhorn iterations per second at d=100.

Workload (one "step"): 1024 pairs of synthetic diagrams (50..500 points each,
birth ~ U[0,1), death = min(birth + Exp(0.2), 1), seed 0), discretised on the
100 x 100 grid plus the diagonal bin, then Algorithm 1 with gamma = 1e-3 until
the marginal L1 error / mass <= 1e-3, and the Sinkhorn cost of Proposition 3.
Points are resident on the GPU before timing starts.

``value`` is pair-iterations per second of the BF16-contraction path with FP32
refinement (every executed iteration counted, BF16 and FP32); the FP32 path on
the same workload is reported beside it.  Kernel durations come from HIP events
on the launch stream; the roofline uses algorithmic flops: 8 d^3 per
pair-iteration (two K applications of two d x d x d contractions each; the
marginal-error check reuses the next application's K v) and 8 d^3 per pair for
the four contractions of the cost, against the 2.5 PFLOP/s dense BF16 peak.

The CPU baseline times the FP64 oracle (dense (d^2+1)-point Sinkhorn) on a
bounded sample of the same pairs.  Only one GPU is used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_BF16 = 2.5e15      # MI355X dense BF16 MFMA, FLOP/s
PEAK_FP32 = 157.3e12    # MI355X FP32 (matrix and vector), FLOP/s
PEAK_HBM = 8.0e12       # B/s

D, GAMMA, TOL, NPAIRS = 100, 1e-3, 1e-3, 1024


def flops_of(iters_total: int, n_pairs: int, d: int = D) -> float:
    """Algorithmic flops of one launch: 8 d^3 per pair-iteration and 8 d^3 per
    pair for the cost (Proposition 3's four contractions).  d, not the padded
    grid; no credit for the skipped triangles; the K application that measures
    the final marginal error is not counted (the paper's loop reuses it)."""
    return 8.0 * d ** 3 * (iters_total + n_pairs)


def run_gpu(precision: str, steps: int, warmup: int, pts_d, off_d, switch_tol: float, gamma: float = GAMMA,
            max_iter: int = 5000, kernel: str = "auto", graph: bool = False):
    import torch
    import paper_1805_08331_amd as pds

    ctx = pds.Context(D, gamma, tol=TOL, max_iter=max_iter, precision=precision, switch_tol=switch_tol,
                      kernel=kernel)
    dev = ctx.device
    n = NPAIRS
    hist = torch.empty((2 * n, D, D), dtype=torch.float32, device=dev)
    mass = torch.empty((2 * n,), dtype=torch.float64, device=dev)
    nbad = torch.zeros((1,), dtype=torch.int32, device=dev)
    ia = torch.arange(0, n, dtype=torch.int32, device=dev)
    ib = torch.arange(n, 2 * n, dtype=torch.int32, device=dev)
    out = pds.DistResult(torch.empty(n, dtype=torch.float64, device=dev),
                         torch.empty((n, 2), dtype=torch.int32, device=dev),
                         torch.empty(n, dtype=torch.float32, device=dev),
                         torch.empty(n, dtype=torch.int32, device=dev))
    ws = ctx.workspace(pds._lib.PDSINK_OP_DIST, n)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]

    def step(i=None):
        pds.pd_discretize(ctx, pts_d, off_d, hist, mass, nbad)
        if i is not None:
            ev[i][0].record(stream)
        pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ib, out=out, ws=ws, check_indices=False)
        if i is not None:
            ev[i][1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for i in range(steps):
        s0 = time.perf_counter()
        step(i)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    iters = out.iters.cpu().numpy().astype(np.int64)
    status = out.status.cpu().numpy()
    cost = out.cost.cpu().numpy()
    err = out.err.cpu().numpy()
    graph_rec = None
    if graph:
        # the same step (discretise + solve) captured once in a HIP graph and
        # replayed: every replay must give the eager step's results bit for bit
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        same = True
        gms = []
        for _ in range(max(steps, 3)):
            out.cost.fill_(-1.0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.replay()
            e1.record(stream)
            e1.synchronize()
            gms.append(e0.elapsed_time(e1))
            same = same and np.array_equal(out.cost.cpu().numpy(), cost) and \
                np.array_equal(out.iters.cpu().numpy().astype(np.int64), iters)
        graph_rec = {"ms_per_step": float(np.median(gms)), "replays": len(gms), "equal_to_eager": bool(same),
                     "of": "discretise + Algorithm 1 + cost, one HIP graph per step"}
        del g
    ctx.close()
    it_total = int(iters.sum())
    return {
        "wall_s": wall,
        "step_ms": step_ms,
        "kernel_ms": kern_ms,
        "iters_total": it_total,
        "iters_bf16": int(iters[:, 0].sum()),
        "iters_fp32": int(iters[:, 1].sum()),
        "n_bad_status": int((status != 0).sum()),
        "max_err": float(err.max()),
        "iters_per_pair": iters.sum(axis=1),
        "status": status,
        "cost": cost,
        "iters_q": {"p50": int(np.percentile(iters.sum(axis=1), 50)),
                    "p99": int(np.percentile(iters.sum(axis=1), 99))},
        "graph": graph_rec,
    }


def cpu_baseline(budget_s: float = 20.0):
    """FP64 oracle on pairs 0, 1, ... of the benchmark batch until ~budget_s of CPU work."""
    import pdgen
    from oracle import ground, sinkhorn
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    d1, d2 = pdgen.pairs_batch(0, 16)
    C = ground.dense_cost(D)
    its, t_used, done = 0, 0.0, 0
    costs = []
    for q in range(16):
        h1, h2 = ground.discretize(d1[q], D), ground.discretize(d2[q], D)
        t0 = time.perf_counter()
        r = sinkhorn.sinkhorn(h1, h2, GAMMA, tol=TOL, max_iter=5000, C=C)
        t_used += time.perf_counter() - t0
        its += r.iters
        costs.append(r.cost)
        done += 1
        if t_used >= budget_s:
            break
    return costs, {"value": its / t_used, "unit": "pair-it/s", "cores": int(blas_threads), "kind": "oracle",
            "sample": f"benchmark batch (1024 pairs, d=100) pairs 0..{done - 1} ({its} pair-iterations, {t_used:.1f} s), FP64 dense "
                      f"(d^2+1)-point kernel on the host, cost matrix built once outside the timing; "
                      f"os.cpu_count()={os.cpu_count()}"}


def cpu_separable(budget_s: float = 8.0, n_pairs: int = 3) -> dict:
    """A second CPU figure: the same alternating iteration and stopping rule
    with K applied in the separable form of Proposition 2, in the log domain
    (FP64 NumPy; at gamma = 1e-3 the 1-D kernel entries underflow FP64, so
    the scalings are kept as logarithms): log(K x) over the grid is two
    log-sum-exp contractions over d, O(d^3) per half step, plus the diagonal
    bin.  Not the oracle (which applies the dense (d^2+1)^2 kernel); timed on
    the first pairs of the benchmark batch until ``budget_s``, iteration
    counts reported to compare with the oracle's."""
    import pdgen
    from scipy.special import logsumexp

    x = np.arange(D, dtype=np.float64)
    G = -((np.abs(x[:, None] - x[None, :]) / D) ** 2) / GAMMA             # log k
    GD = -2.0 * ((np.abs(x[None, :] - x[:, None]) / (2 * D)) ** 2) / GAMMA  # log k_Delta at cell (i, j)

    def log_k(LX, lxd):
        T = logsumexp(G[None, :, :] + LX[:, None, :], axis=2)      # T[k, j] = LSE_l G[j, l] + LX[k, l]
        W = logsumexp(G[:, :, None] + T[None, :, :], axis=1)       # W[i, j] = LSE_k G[i, k] + T[k, j]
        return np.logaddexp(W, lxd + GD), np.logaddexp(logsumexp(LX + GD), lxd)

    def hist(pts):
        h = np.zeros((D, D))
        ij = np.minimum(np.floor(pts.astype(np.float64) * D).astype(np.int64), D - 1)
        np.add.at(h, (ij[:, 0], ij[:, 1]), 1.0)
        return h

    d1, d2 = pdgen.pairs_batch(0, n_pairs)
    its, t_used, counts = 0, 0.0, []
    with np.errstate(divide="ignore", invalid="ignore"):
        for q in range(n_pairs):
            A, B = hist(d1[q]), hist(d2[q])
            ma, mb = A.sum(), B.sum()
            la, lb = np.log(A), np.log(B)
            lad, lbd = np.log(mb), np.log(ma)                       # Proposition 1: a_Delta = |b|, b_Delta = |a|
            m = ma + mb
            LV, lvd = np.zeros((D, D)), 0.0
            t0 = time.perf_counter()
            done = False
            for t in range(1, 5001):
                KV, kvd = log_k(LV, lvd)
                LU, lud = la - KV, lad - kvd
                KU, kud = log_k(LU, lud)
                LV, lvd = lb - KU, lbd - kud
                KV2, kvd2 = log_k(LV, lvd)
                err = (np.nansum(np.abs(np.exp(LU + KV2) - A)) + abs(np.exp(lud + kvd2) - mb)) / m
                its += 1
                if err <= TOL:
                    done = True
                    break
                if t_used + time.perf_counter() - t0 >= budget_s:
                    break
            t_used += time.perf_counter() - t0
            if done:
                counts.append(t)
            if t_used >= budget_s:
                break
    return {"value": its / t_used, "unit": "pair-it/s", "cores": 1, "kind": "cpu separable (log domain, FP64)",
            "iterations_to_tol": counts,
            "sample": f"benchmark batch from pair 0: {its} pair-iterations in {t_used:.1f} s, pairs run to "
                      f"tol {TOL} took {counts} iterations (the oracle: 157, 495, 348); each iteration also "
                      f"applies K once more for the error check"}


def pmc_probe(pts_d, off_d, switch_tol: float, copy_mib: int = 256):
    """One BF16 batch and one plain device copy of known size, for counter runs
    (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE): the copy calibrates the
    counters' byte scale."""
    import torch
    import paper_1805_08331_amd as pds

    ctx = pds.Context(D, GAMMA, tol=TOL, max_iter=5000, precision="bf16", switch_tol=switch_tol)
    hist, mass, nbad = pds.pd_discretize(ctx, pts_d, off_d)
    n = NPAIRS
    ia = torch.arange(0, n, dtype=torch.int32, device=ctx.device)
    ib = torch.arange(n, 2 * n, dtype=torch.int32, device=ctx.device)
    pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ib)
    src = torch.ones(copy_mib << 18, dtype=torch.float32, device=ctx.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"pmc_probe": True, "copy_bytes": copy_mib << 20, "pairs": n}))


PHASE_NAMES = ["setup", "scale_normalisers", "bf16_kernel_build", "contraction_1", "contraction_2",
               "update_first_pass", "suspects", "refit", "update_final_pass", "cost"]
COUNT_NAMES = ["half_steps", "refits", "kernel_builds", "normaliser_computations", "half_steps_with_suspects",
               "pairs"]


def phase_profile(pts_d, off_d, switch_tol: float, precision: str = "bf16"):
    """One batch through the instrumented library (libpdsink_prof.so): cycles
    of each phase of the resident-kernel solve, summed over the pairs, as
    seen by the first wave of each workgroup between workgroup barriers."""
    import ctypes
    import torch
    import paper_1805_08331_amd as pds

    lib = pds._lib.load()
    if pds._lib.LIB_NAME != "libpdsink_prof.so":
        raise SystemExit("--phases needs the instrumented build (python -m paper_1805_08331_amd.build --profile)")
    ctx = pds.Context(D, GAMMA, tol=TOL, max_iter=5000, precision=precision, switch_tol=switch_tol)
    hist, mass, nbad = pds.pd_discretize(ctx, pts_d, off_d)
    n = NPAIRS
    ia = torch.arange(0, n, dtype=torch.int32, device=ctx.device)
    ib = torch.arange(n, 2 * n, dtype=torch.int32, device=ctx.device)
    buf = (ctypes.c_uint64 * 16)()
    pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ib)
    pds._lib.check("pdsink_phase_profile", lib.pdsink_phase_profile(buf, 1))
    r = pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ib)
    pds._lib.check("pdsink_phase_profile", lib.pdsink_phase_profile(buf, 0))
    iters = int(r.iters.sum().item())
    ctx.close()
    cyc = [int(buf[k]) for k in range(len(PHASE_NAMES))]
    cnt = {name: int(buf[len(PHASE_NAMES) + k]) for k, name in enumerate(COUNT_NAMES)}
    tot = sum(cyc)
    print(json.dumps({"phases": {nm: {"cycles": c, "share": c / tot, "per_pair_iteration": c / max(iters, 1)}
                                 for nm, c in zip(PHASE_NAMES, cyc)},
                      "counts": cnt, "pair_iterations": iters, "cycles_per_pair_iteration": tot / max(iters, 1),
                      "precision": precision,
                      "workload": f"{NPAIRS} pairs, d={D}, gamma={GAMMA}, tol={TOL}, switch_tol={switch_tol}"}),
          flush=True)


# The translation unit of the plain pair kernel and what it includes (the
# bounds variant and the log-domain path are compiled in units of their own).
PAIR_KERNEL_SOURCES = ("pdsink_api.hip", "pdsink_device.h", "sinkhorn_log.h", "sinkhorn_pair.h", "sinkhorn_fast.h")
PAIR_KERNEL_NAME = "sinkhorn_fast_kernel"


def source_hash() -> str:
    """Hash of the pair kernel's sources: counter figures apply only to the build they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1805_08331_amd", "csrc")
    for name in PAIR_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the pair kernel from the committed counter summary,
    or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "sinkhorn_fast_kernel_d100_1024pairs_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    return rec.get("traffic_bytes") if rec.get("source_hash") == source_hash() else None


def write_traffic(fetch_csv: str, write_csv: str, out: str | None = None):
    """Summarise two rocprofv3 counter runs of ``--pmc-probe`` (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) into the traffic record of the pair kernel,
    scaled by what the counters read for the 256 MiB calibration copy."""
    import csv

    def rows(path, counter):
        with open(path, newline="") as fh:
            return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
                    for r in csv.DictReader(fh) if r["Counter_Name"] == counter]

    fr, wr = rows(fetch_csv, "FETCH_SIZE"), rows(write_csv, "WRITE_SIZE")
    if len(fr) != len(wr):
        raise SystemExit("the two counter runs saw different dispatch lists")
    copy_bytes = 256 << 20
    copy = [i for i, (n, g, v) in enumerate(fr) if n.startswith("__amd_rocclr_copyBuffer")]
    ci = max(copy, key=lambda i: fr[i][2])
    kern = [i for i, (n, g, v) in enumerate(fr) if PAIR_KERNEL_NAME in n and g == NPAIRS * 512]
    if len(kern) != 1:
        raise SystemExit("expected one level-0 launch of the pair kernel")
    ki = kern[0]
    ff = copy_bytes / 1024 / fr[ci][2]
    wf = copy_bytes / 1024 / wr[ci][2]
    traffic = (fr[ki][2] * ff + wr[ki][2] * wf) * 1024
    rec = {"kernel": PAIR_KERNEL_NAME,
           "workload": "1024 PD pairs, d=100, gamma=1e-3, tol=1e-3, BF16+FP32 refinement",
           "source_hash": source_hash(), "fetch_kib_raw": fr[ki][2], "write_kib_raw": wr[ki][2],
           "copy_calibration": {"bytes": copy_bytes, "fetch_kib_raw": fr[ci][2], "write_kib_raw": wr[ci][2],
                                "fetch_factor": ff, "write_factor": wf},
           "traffic_bytes": int(round(traffic)),
           # two d x d FP32 histograms per pair in; cost, 2 iteration counts, error, status, route byte out
           "algorithmic_bytes": NPAIRS * (2 * 100 * 100 * 4 + 8 + 8 + 4 + 4 + 1)}
    if out is None:
        out = os.path.join(ROOT, "profiles", "sinkhorn_fast_kernel_d100_1024pairs_traffic.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print("| dispatch | grid | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) |")
    print("|---|---|---|---|")
    for (n, g, v), (_, _, w) in zip(fr, wr):
        if n.startswith("__amd_rocclr_copyBuffer") and g < 1 << 16:
            continue
        short = n.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0][:60]
        print(f"| `{short}` | {g} | {v:.1f} | {w:.1f} |")
    print(json.dumps(rec))


def gamma_sweep(pts_d, off_d, switch_tol: float):
    """The benchmark batch (BF16 + refinement) at gamma_n = 0.1 / n, n = 1 ... 5000
    (down to 2e-5): iterations, throughput and the paths the pairs took, one
    JSON line per gamma."""
    for n in (1, 10, 100, 200, 500, 1000, 2000, 5000):
        g = 0.1 / n
        for prec in ("bf16",):
            r = run_gpu(prec, 1, 1, pts_d, off_d, switch_tol, gamma=g, max_iter=40000)
            st = r["status"]
            print(json.dumps({
                "gamma": g, "gamma_d2": g * D * D, "precision": prec, "pairs": NPAIRS,
                "pair_iters": r["iters_total"], "kernel_ms": float(np.mean(r["kernel_ms"])),
                "pair_it_per_s": r["iters_total"] / (float(np.mean(r["kernel_ms"])) / 1e3),
                "iters_p50": r["iters_q"]["p50"], "iters_p99": r["iters_q"]["p99"],
                "converged": int((st == 0).sum()), "log_path": int(((st & 8) != 0).sum()),
                "flagged": int(((st & 6) != 0).sum()), "max_iter": int(((st & 1) != 0).sum())}), flush=True)


def scaling_study(n_pairs: int = 64, ns=(10, 20, 50, 100, 200, 500, 1000, 2000, 5000), max_iter: int = 40000,
                  large_pairs: int = 16):
    """Distance time against diagram size at gamma_n = 0.1 / n (the scaling
    experiment of section 5): for each n, ``n_pairs`` pairs of random diagrams
    of n to 2n points, d = 100, BF16 contractions with FP32 refinement to
    marginal error 1e-3 (pairs beyond the scaled representation's range go
    to the log-domain path).  One JSON line per n, with the batch time, the
    iteration quantiles, the paths the pairs took and t_n / t_10.  From
    n = 1000 on the batch has ``large_pairs`` pairs (they run side by side, so
    the batch time is that of its slowest pair); only the first n has an
    untimed warm-up launch."""
    import torch
    import pdgen
    import paper_1805_08331_amd as pds

    t10 = None
    for n in ns:
        g = 0.1 / n
        npairs = n_pairs if n < 1000 else large_pairs
        print(f"scaling: n = {n}, {npairs} pairs", file=sys.stderr, flush=True)
        d1, d2 = pdgen.pairs_batch(n, npairs, n, 2 * n)
        pts, off = pdgen.to_csr(d1 + d2)
        with pds.Context(D, g, tol=TOL, max_iter=max_iter, precision="bf16", switch_tol=0.8e-3) as ctx:
            hist, _, _ = pds.pd_discretize(ctx, torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda())
            ia = torch.arange(0, npairs, dtype=torch.int32, device=hist.device)
            ws = ctx.workspace(pds._lib.PDSINK_OP_DIST, npairs)
            out = pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ia + npairs, ws=ws) if t10 is None else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = pds.sinkhorn_dist_batch(ctx, hist, hist, ia, ia + npairs, out=out, ws=ws, check_indices=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            supp = (hist > 0).sum(dim=(1, 2)).cpu().numpy()
        it = out.iters.sum(dim=1).cpu().numpy()
        st = out.status.cpu().numpy()
        t10 = ms if t10 is None else t10
        print(json.dumps({
            "n": n, "points": f"{n}-{2 * n}", "gamma": g, "gamma_d2": g * D * D, "pairs": npairs, "batch_ms": ms,
            "ms_per_pair": ms / npairs, "t_over_t10": ms / t10,
            "iters_p50": int(np.percentile(it, 50)), "iters_p99": int(np.percentile(it, 99)),
            "support_max": int(supp.max()), "converged": int(((st & 7) == 0).sum()),
            "log_path": int(((st & 8) != 0).sum()), "flagged": int(((st & 6) != 0).sum()),
            "max_iter": int(((st & 1) != 0).sum())}), flush=True)


def kmeans_bench(rounds: int = 2, n_diag: int = 4000, k: int = 10, d: int = 100, gamma: float = GAMMA,
                 max_outer: int = 10, sharpen: bool = False):
    """The k-means workload: ``n_diag`` diagrams drawn around 10 templates of
    200 points (jitter 0.03, +-20 % points), k = 10, d = 100, BF16 with FP32
    refinement to marginal error 1e-3.  Lloyd rounds run through the binding's
    calls (assignment of all n_diag x k pairs, then the barycenter of each
    cluster's members from the uniform start, at most ``max_outer`` outer
    steps, energy rtol 0.01), one JSON line per round with its timings.
    ``sharpen``: each barycenter is then sharpened (pd_sharpen) to the mean
    entropy of its members' histograms, the use the paper suggests for its
    smeared barycenters."""
    import torch
    import pdgen
    import paper_1805_08331_amd as pds

    diags, labels = pdgen.kmeans_set(0, n_diag)
    pts, off = pdgen.to_csr(diags)
    init = np.random.default_rng(0).choice(n_diag, size=k, replace=False)
    with pds.Context(d, gamma, tol=TOL, max_iter=5000, precision="bf16", switch_tol=0.8e-3) as ctx:
        hist, _, _ = pds.pd_discretize(ctx, torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda())
        cents = hist[torch.from_numpy(init).cuda().long()].contiguous()
        ws = ctx.workspace(pds._lib.PDSINK_OP_KMEANS, n_diag * k)
        for r in range(rounds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            assign, dist, st = pds.kmeans_assign(ctx, hist, cents, ws=ws)
            torch.cuda.synchronize()
            t_assign = time.perf_counter() - t0
            a = assign.cpu().numpy()
            obj = float(dist.cpu().numpy()[np.arange(n_diag), a].sum())
            t1 = time.perf_counter()
            outer = []
            for c in range(k):
                members = np.nonzero(a == c)[0]
                if members.size == 0:
                    continue
                mh = hist[torch.from_numpy(members).cuda().long()].contiguous()
                z, _, n_out = pds.pd_barycenter(ctx, mh, lam=5.0, max_outer=max_outer, energy_rtol=0.01)
                if sharpen:
                    p = mh.reshape(members.size, -1).double().cpu().numpy()
                    p = p / p.sum(axis=1, keepdims=True)
                    h0 = float(np.mean(-np.sum(np.where(p > 0, p * np.log(np.where(p > 0, p, 1.0)), 0.0), axis=1)))
                    pds.pd_sharpen(ctx, z, h0)
                cents[c] = z
                outer.append(n_out)
            torch.cuda.synchronize()
            t_bary = time.perf_counter() - t1
            # purity: the share of diagrams in the majority template of their cluster
            purity = sum(int(np.bincount(labels[a == c], minlength=k).max()) for c in range(k) if np.any(a == c))
            purity /= n_diag
            print(json.dumps({
                "round": r, "assign_s": t_assign, "assign_pairs_per_s": n_diag * k / t_assign,
                "barycenters_s": t_bary, "outer_steps": outer, "objective": obj,
                "bad_status": int(np.count_nonzero(st.cpu().numpy() & 6)),
                "purity": purity, "sharpened": sharpen,
                "workload": f"{n_diag} diagrams, k={k}, d={d}, gamma={gamma}, BF16 + FP32 refinement, tol {TOL}"}),
                flush=True)


def serve_bench(seconds: float, rate: float = 2000.0, k: int = 10, slots: int = 16, max_pairs: int = 512,
                mem_budget: int = 64 << 30):
    """Serving loop on a Poisson stream: ``rate`` requests/s for ``seconds``
    (after a 1 s warm-up stream), half distances and half assignments to k
    resident centroids, grids 50, 100 and 200, lognormal(5, 0.7) point counts;
    gamma = 1e-3, stop at marginal error 1e-3.  Prints one JSON line with the
    latency percentiles (arrival to result on the host) and the throughput."""
    import torch
    import pdgen
    import paper_1805_08331_amd as pds
    from paper_1805_08331_amd import serve

    grids = (50, 100, 200)
    cdiags, _ = pdgen.kmeans_set(1, k, n_templates=k)
    cents = {}
    for d in grids:
        with pds.Context(d, GAMMA) as ctx:
            pts, off = pdgen.to_csr(cdiags)
            h, _, _ = pds.pd_discretize(ctx, torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda())
            torch.cuda.synchronize()
            cents[d] = h.contiguous()
    # tiling of each grid's distance kernel, timed on 256 pairs drawn like the
    # stream's (the choice is cached for the server's contexts)
    from paper_1805_08331_amd import autotune
    tiling = {}
    for d in grids:
        if d not in autotune.RESIDENT_GRIDS:
            tiling[str(d)] = {"kernel": "general (the only tiling at this grid)"}
            continue
        sd1, sd2 = pdgen.pairs_batch(100 + d, 256, 20, 600)
        with pds.Context(d, GAMMA) as ctx:
            pts, off = pdgen.to_csr(sd1 + sd2)
            h, _, _ = pds.pd_discretize(ctx, torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda())
        ia = torch.arange(0, 256, dtype=torch.int32, device=h.device)
        t = autotune.tune_kernel(h, h, ia, ia + 256, d, GAMMA, TOL, precision="bf16", switch_tol=0.8e-3, reps=2)
        tiling[str(d)] = {"kernel": t["kernel"], "median_ms": t["median_ms"]}
    print(f"serve: kernel tiling {tiling}", file=sys.stderr, flush=True)
    srv = serve.Server(grids, GAMMA, centroids=cents, slots=slots, max_pairs=max_pairs, mem_budget=mem_budget,
                       tol=TOL, max_iter=5000, precision="bf16", switch_tol=0.8e-3)
    serve.run_stream(srv, pdgen.serve_stream(1, rate=rate, duration=1.0, grids=grids), timeout_s=120)
    print("serve: warm-up done", file=sys.stderr, flush=True)
    stream = pdgen.serve_stream(0, rate=rate, duration=seconds, grids=grids)
    srv.peak_bytes = 0
    n0 = srv.n_launches
    reqs, wall = serve.run_stream(srv, stream, timeout_s=seconds * 10 + 60)
    n_launch = srv.n_launches - n0
    srv.close()
    lat = serve.latency_summary([r.latency for r in reqs])
    by_grid = {str(d): serve.latency_summary([r.latency for r in reqs if r.d == d]) for d in grids}
    by_kind = {name: serve.latency_summary([r.latency for r in reqs if r.kind == kind])
               for name, kind in (("distance", serve.DIST), ("assign", serve.ASSIGN))}
    n_pairs = sum(r.n_pairs(k) for r in reqs)
    bad = sum(int(np.count_nonzero(r.status & ~8)) for r in reqs)
    log_path = {str(d): sum(int(np.count_nonzero(r.status & 8)) for r in reqs if r.d == d) for d in grids}
    print(json.dumps({
        "metric": "serving latency, arrival to result on the host", "unit": "ms",
        "p50_ms": lat["p50_ms"], "p99_ms": lat["p99_ms"], "max_ms": lat["max_ms"],
        "requests": len(reqs), "offered_req_per_s": rate, "duration_s": seconds,
        "served_req_per_s": len(reqs) / wall, "pairs_per_s": n_pairs / wall, "bad_status_pairs": bad, "log_path_pairs": log_path,
        "peak_device_bytes": srv.peak_bytes, "launches": n_launch, "by_grid": by_grid, "by_kind": by_kind,
        "kernel_tiling": tiling,
        "config": {"workload": "Poisson stream, half distances and half k-means assignments (k resident "
                               "centroids), d uniform in {50, 100, 200}, lognormal(5, 0.7) points",
                   "k": k, "gamma": GAMMA, "tol": TOL, "slots": slots, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                   "max_pairs_per_launch": max_pairs, "mem_budget_bytes": mem_budget,
                   "precision": "bf16 contractions, fp32 refinement"},
        "data": "synthetic"}), flush=True)


def bary_bench(outer: int = 3, n_diag: int = 256, d: int = 200, gamma: float = 2e-3, tol: float = 1e-4,
               switch_tol: float = 1e-3) -> dict:
    """The barycenter workload: ``n_diag`` perturbations of one template
    (100-400 points, jitter 0.02, 10 % fresh points), d = 200, gamma = 2e-3,
    BF16 contractions with FP32 refinement, inner solves to marginal error
    ``tol``, warm-started between steps.  After one untimed step, ``outer``
    steps of Algorithm 2 from the uniform start are timed end to end (the outer
    loop synchronises with the host once per step, for its stopping test)."""
    import torch
    import pdgen
    import paper_1805_08331_amd as pds

    diags = pdgen.bary_set(0, n_diag=n_diag)
    pts, off = pdgen.to_csr(diags)
    with pds.Context(d, gamma, tol=tol, max_iter=20000, precision="bf16", switch_tol=switch_tol) as ctx:
        hist, _, _ = pds.pd_discretize(ctx, torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda())
        ws = ctx.workspace(pds._lib.PDSINK_OP_BARYCENTER, n_diag)
        pds.pd_barycenter(ctx, hist, lam=5.0, max_outer=1, energy_rtol=0.0, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z, energy, n_out = pds.pd_barycenter(ctx, hist, lam=5.0, max_outer=outer, energy_rtol=0.0, ws=ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    return {"ms_per_outer_step": wall / n_out * 1e3, "outer_steps": n_out, "energy": energy,
            "config": {"workload": f"barycenter of {n_diag} diagrams (100-400 points, one template, jitter 0.02, "
                                   f"10% fresh points), d={d} grid + diagonal bin, gamma={gamma}",
                       "precision": "bf16 contractions, fp32 refinement", "inner_tol": tol, "switch_tol": switch_tol,
                       "lambda": 5.0}}


def serve_leg(seconds: float = 3.0, rate: float = 2000.0) -> dict:
    """The serving loop (serve_bench) in a child process, which sets its own
    number of hardware queues before HIP starts: its JSON line, parsed."""
    import subprocess
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--serve", str(seconds), "--serve-rate", str(rate)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=seconds * 10 + 240)
    if r.returncode != 0:
        return {"error": f"exit {r.returncode}: {r.stderr.strip().splitlines()[-1:]}"}
    line = [x for x in r.stdout.splitlines() if x.startswith("{")][-1]
    rec = json.loads(line)
    return {k: rec[k] for k in ("p50_ms", "p99_ms", "max_ms", "requests", "offered_req_per_s", "served_req_per_s",
                                "pairs_per_s", "bad_status_pairs", "by_grid", "kernel_tiling", "config")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["bf16", "fp32"], default=None, help="run one precision only")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run one BF16 batch and a 256 MiB device copy (for counter runs), then exit")
    ap.add_argument("--switch-tol", type=float, default=0.8e-3,
                    help="BF16 -> FP32 switch point of the marginal error (0.8 x tol: the shortest batch time)")
    ap.add_argument("--gamma-sweep", action="store_true",
                    help="run the batch at gamma = 0.1 / n down to 2e-5 and print one line per gamma, then exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record from two --pmc-probe counter runs, then exit")
    ap.add_argument("--autotune", action="store_true",
                    help="time the benchmark batch at several BF16 -> FP32 switch points, print the choice, then exit")
    ap.add_argument("--serve", type=float, metavar="SECONDS", default=None,
                    help="run the serving loop on a Poisson stream for SECONDS and print its latency line, then exit")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="offered requests per second (--serve)")
    ap.add_argument("--serve-slots", type=int, default=16, help="launch slots, shared by all grids (--serve)")
    ap.add_argument("--serve-hw-queues", type=int, default=16,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before HIP starts; --serve)")
    ap.add_argument("--serve-max-pairs", type=int, default=512, help="pairs per launch at most (--serve)")
    ap.add_argument("--kmeans", type=int, metavar="ROUNDS", default=None,
                    help="Lloyd rounds of the k-means workload (4000 diagrams, k = 10, d = 100), then exit")
    ap.add_argument("--kmeans-sharpen", action="store_true",
                    help="with --kmeans: sharpen each barycenter to its members' mean entropy")
    ap.add_argument("--scaling", action="store_true",
                    help="distance time against diagram size n at gamma = 0.1 / n (n = 10 ... 5000), then exit")
    ap.add_argument("--bary", type=int, metavar="STEPS", default=None,
                    help="time STEPS outer steps of the barycenter workload, print its line, then exit")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the barycenter and serving legs of the default line")
    ap.add_argument("--phases", choices=["bf16", "fp32"], default=None,
                    help="phase cycle split of one batch through the instrumented library, then exit")
    args = ap.parse_args()
    if args.phases:
        os.environ["PDSINK_PROFILE_BUILD"] = "1"   # read when the package loads the library
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the per-GPU shard is the batch measured at --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.serve is not None:
        if not 1 <= args.serve_hw_queues <= 16:
            print("--serve-hw-queues must be in 1..16", file=sys.stderr)
            sys.exit(2)
        # read by the HIP runtime when it starts (torch is not imported yet)
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_hw_queues)
        serve_bench(args.serve, rate=args.serve_rate, slots=args.serve_slots, max_pairs=args.serve_max_pairs)
        return

    import torch
    import pdgen

    d1, d2 = pdgen.pairs_batch(0, NPAIRS)
    pts, off = pdgen.to_csr(d1 + d2)
    pts_d = torch.from_numpy(pts).cuda()
    off_d = torch.from_numpy(off).cuda()

    if args.pmc_probe:
        pmc_probe(pts_d, off_d, args.switch_tol)
        return
    if args.bary is not None:
        print(json.dumps(bary_bench(args.bary)), flush=True)
        return
    if args.scaling:
        scaling_study()
        return
    if args.kmeans is not None:
        kmeans_bench(args.kmeans, sharpen=args.kmeans_sharpen)
        return
    if args.phases:
        phase_profile(pts_d, off_d, args.switch_tol, args.phases)
        return
    if args.gamma_sweep:
        gamma_sweep(pts_d, off_d, args.switch_tol)
        return
    if args.autotune:
        import paper_1805_08331_amd as pds
        from paper_1805_08331_amd import autotune
        with pds.Context(D, GAMMA) as ctx:
            hist, _, _ = pds.pd_discretize(ctx, pts_d, off_d)
        ia = torch.arange(0, NPAIRS, dtype=torch.int32, device=hist.device)
        r = autotune.tune_switch_tol(hist, hist, ia, ia + NPAIRS, D, GAMMA, TOL, reps=5)
        print(json.dumps({"autotune": "switch_tol", "workload": f"{NPAIRS} pairs, d={D}, gamma={GAMMA}, tol={TOL}",
                          "switch_tol": r["switch_tol"],
                          "median_ms": {f"{k:.3g}": float(np.median(v)) for k, v in r["ms"].items()},
                          "iters_bf16_fp32": {f"{k:.3g}": v for k, v in r["iters"].items()}}), flush=True)
        return

    res = {}
    # tiling of the distance kernel: timed on the benchmark batch itself, the
    # faster one runs the timed steps (both solve the same iteration)
    import paper_1805_08331_amd as pds
    from paper_1805_08331_amd import autotune
    with pds.Context(D, GAMMA) as ctx:
        hist_t, _, _ = pds.pd_discretize(ctx, pts_d, off_d)
    ia_t = torch.arange(0, NPAIRS, dtype=torch.int32, device=hist_t.device)
    tuned = {}
    for prec in (["bf16", "fp32"] if args.only is None else [args.only]):
        t = autotune.tune_kernel(hist_t, hist_t, ia_t, ia_t + NPAIRS, D, GAMMA, TOL, precision=prec,
                                 switch_tol=args.switch_tol, reps=3)
        tuned[prec] = {"kernel": t["kernel"], "median_ms": t["median_ms"], "cost_rel": t["cost_rel"]}
        print(f"[{prec}] kernel tiling: {t['median_ms']} -> {t['kernel']}", file=sys.stderr, flush=True)
    del hist_t
    for prec in (["bf16", "fp32"] if args.only is None else [args.only]):
        r = run_gpu(prec, args.steps, args.warmup, pts_d, off_d, args.switch_tol, kernel=tuned[prec]["kernel"],
                    graph=prec == "bf16")
        k_avg = float(np.mean(r["kernel_ms"])) / 1e3
        fl = flops_of(r["iters_total"], NPAIRS)
        r["pair_it_per_s"] = r["iters_total"] * args.steps / r["wall_s"]
        r["kernel_pair_it_per_s"] = r["iters_total"] / k_avg
        r["pairs_per_s"] = NPAIRS * args.steps / r["wall_s"]
        r["achieved_tflops"] = fl / k_avg / 1e12
        if prec == "bf16":
            # the dense BF16 peak; beside it, the peak of this mix of BF16 and
            # FP32 contractions (the refinement and the cost run in FP32)
            f_b = 8.0 * D ** 3 * r["iters_bf16"]
            f_f = fl - f_b
            peak = PEAK_BF16
            r["peak_blend_tflops"] = fl / (f_b / PEAK_BF16 + f_f / PEAK_FP32) / 1e12
        else:
            peak = PEAK_FP32
        r["peak_tflops"] = peak / 1e12
        res[prec] = r
        ipp = r.pop("iters_per_pair")
        r["iters_quantiles"] = {"p50": int(np.percentile(ipp, 50)), "p99": int(np.percentile(ipp, 99)),
                                "max": int(ipp.max())}
        print(f"[{prec}] {r['iters_total']} pair-iterations per step, kernel {k_avg * 1e3:.2f} ms, "
              f"{r['kernel_pair_it_per_s']:.3e} pair-it/s, {r['achieved_tflops']:.1f} TFLOP/s, "
              f"bad status {r['n_bad_status']}, iterations per pair {r['iters_quantiles']} "
              f"(bf16 {r['iters_bf16']}, fp32 {r['iters_fp32']})",
              file=sys.stderr, flush=True)

    main_key = "bf16" if "bf16" in res else "fp32"
    m = res[main_key]
    k_avg = float(np.mean(m["kernel_ms"])) / 1e3
    out = {
        "metric": "PD-pair Sinkhorn iters/sec at d=100, bf16 vs fp32 @1e-3 err; p50/p99 latency",
        "value": m["pair_it_per_s"],
        "unit": "pair-it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if main_key == "bf16" else "fp32",
        "data": "synthetic",
        "config": {"workload": "batched distances: 1024 PD pairs, 50-500 points, d=100 grid + diagonal bin, "
                               "gamma=1e-3, stop at marginal L1 error 1e-3",
                   "pairs": NPAIRS, "d": D, "gamma": GAMMA, "tol": TOL,
                   "precision": "bf16 contractions, fp32 refinement" if main_key == "bf16" else "fp32",
                   "switch_tol": args.switch_tol},
        "pairs_per_s": m["pairs_per_s"],
        "pair_iters_per_step": m["iters_total"],
        "latency_ms": {"p50": float(np.percentile(m["step_ms"], 50)), "p99": float(np.percentile(m["step_ms"], 99)),
                       "of": "one 1024-pair batch (discretise + Algorithm 1 + cost)"},
        "roofline": {"bound": "mfma", "achieved": m["achieved_tflops"], "peak": m["peak_tflops"], "unit": "TFLOP/s",
                     "frac": m["achieved_tflops"] / m["peak_tflops"], "traffic": measured_traffic(),
                     "kernel": PAIR_KERNEL_NAME if tuned[main_key]["kernel"] == "resident" else "sinkhorn_pair_kernel",
                     "kernel_ms": k_avg * 1e3,
                     "flops": "8 d^3 per pair-iteration + 8 d^3 per pair (cost), d = 100"},
    }
    if "peak_blend_tflops" in m:
        out["roofline"]["peak_blend_bf16_fp32"] = m["peak_blend_tflops"]
        out["roofline"]["frac_of_blend"] = m["achieved_tflops"] / m["peak_blend_tflops"]
    if "fp32" in res and main_key == "bf16":
        f = res["fp32"]
        out["fp32"] = {"value": f["pair_it_per_s"], "unit": "pair-it/s", "pair_iters_per_step": f["iters_total"],
                       "kernel_ms": float(np.mean(f["kernel_ms"])), "achieved_tflops": f["achieved_tflops"],
                       "frac_of_fp32_peak": f["achieved_tflops"] / f["peak_tflops"], "pairs_per_s": f["pairs_per_s"]}
        out["bf16_over_fp32"] = m["pair_it_per_s"] / f["pair_it_per_s"]
        out["bf16_iterations"] = {"bf16": m["iters_bf16"], "fp32_refine": m["iters_fp32"]}
        rd = np.abs(m["cost"] - f["cost"]) / np.maximum(np.abs(f["cost"]), 1e-300)
        # both stop at marginal error 1e-3, at different iterates: this is the
        # spread of that stopping rule, not the parity bar (the tests compare
        # BF16 refined to 1e-5 with the converged oracle)
        out["bf16_vs_fp32_cost_rel"] = {"max": float(rd.max()), "median": float(np.median(rd))}
    out["iterations_per_pair"] = m["iters_quantiles"]
    if m.get("graph"):
        out["graph_replay"] = m["graph"]
    out["kernel_tiling"] = {"choice": {k: v["kernel"] for k, v in tuned.items()},
                            "median_ms": {k: v["median_ms"] for k, v in tuned.items()},
                            "cost_rel_between": {k: v["cost_rel"] for k, v in tuned.items()},
                            "candidates": "resident: K depth 16 ceil(d/16) = 112, BF16 kernels cached in LDS; "
                                          "general: grid padded to 128, 32x32 tiles"}
    if not args.no_extra:
        print("barycenter leg", file=sys.stderr, flush=True)
        try:
            out["barycenter"] = bary_bench(3)
        except Exception as e:   # reported in the line, the headline figures stand
            out["barycenter"] = {"error": repr(e)}
        print("serving leg", file=sys.stderr, flush=True)
        out["serving"] = serve_leg()
    if not args.no_cpu:
        oc, out["cpu_baseline"] = cpu_baseline()
        out["cpu_separable"] = cpu_separable()
        n = len(oc)
        for key in res:
            dev = np.abs(res[key]["cost"][:n] - np.array(oc)) / np.abs(np.array(oc))
            out.setdefault("oracle_cost_rel_same_tol", {})[key] = {"pairs": n, "max": float(dev.max())}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
