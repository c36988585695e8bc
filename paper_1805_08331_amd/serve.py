"""Serving loop: continuous batching of distance and assignment requests.

A request is either a distance between two diagrams (Algorithm 1 on one pair)
or an assignment of one diagram to the nearest of k centroids held on the
device (the assignment step of k-means, k pairs).  Requests come at any of
several grid sizes d.  The loop keeps, per grid, one ``Context``, the
resident centroid histograms; all grids share a fixed pool of launch slots,
a slot being a HIP stream (default priority) with at most one launch in
flight.  A launch is one call of ``sinkhorn_dist_batch_notify`` over every
pair of its requests (a distance is one pair, an assignment k pairs against
the grid's centroids), which posts each pair's result to pinned host memory
as soon as that pair is solved: a request completes when its own pairs are
done, not when the slowest pair of its launch is.  The pool should be no
larger than the hardware queues the process gets (``GPU_MAX_HW_QUEUES``, read
when the HIP runtime starts; four by default): streams beyond that share a
queue, and a short launch then waits behind a long one on the same queue.  More queues let more launches overlap:
a slot is free again once its launch has ended, and while it runs the
other slots keep the chip busy.  Each turn of ``Server.poll``:

1. collects results: for every launch in flight, the completion records its
   pairs have posted so far (the tag of a record is stored last, so a tagged
   record is whole); a request whose pairs are all posted gets its results
   and completion time.  A launch whose HIP event has passed (queried without
   blocking) has posted every pair; its slot and memory are released;
2. gives each free slot to the grid whose oldest waiting request is the
   oldest, and admits that grid's waiting requests, oldest first, a request
   whole (its one pair, or its k pairs), up to a pair cap per launch
   and within a device-memory budget counted over all launches in flight;
3. launches the batch on the slot's stream: discretisation of the batch's
   diagrams, a copy of the grid's centroids behind them (assignments), and
   one distance call over all pairs.  Launches in different slots and at
   different grids run on the device at the same time; requests that arrive
   meanwhile wait for the next free slot.

Every pair's arithmetic depends only on its own two histograms (the library
routes and orders pairs by their own supports), so a request's result is the
same served alone or in a mix.

Latency of a request: from its arrival stamp (host clock) to the turn of the
loop that sees its result on the host.

Only host logic lives here; every step of the computation runs in the
library's kernels, through the bindings of this package.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import Context, _lib, autotune, done_records, done_view, pd_discretize, sinkhorn_dist_batch_notify

DIST = 0
ASSIGN = 1


@dataclass
class Request:
    """One query.  ``diagrams`` holds two point arrays (DIST) or one (ASSIGN),
    each float32 [n, 2] of (birth, death) in [0, 1]^2."""
    kind: int
    d: int
    diagrams: list
    t_arrival: float = 0.0
    rid: int = -1
    # results, filled when the request's pairs have posted theirs
    cost: float | None = None          # DIST: Sinkhorn cost
    assign: int | None = None          # ASSIGN: nearest centroid
    dists: np.ndarray | None = None    # ASSIGN: costs to the k centroids
    status: np.ndarray | None = None   # status word(s) of its pair(s)
    t_done: float | None = None

    def n_pairs(self, k: int) -> int:
        return 1 if self.kind == DIST else k

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrival


def plan_batch(waiting, k: int, max_pairs: int, budget: int, req_bytes, ws_bytes) -> list:
    """Requests of one grid for the next launch: the longest prefix of
    ``waiting`` (oldest first) whose pair count stays within ``max_pairs`` and
    whose device bytes stay within ``budget``.  The bytes of a prefix are the
    sum of ``req_bytes(r)`` over its requests plus ``ws_bytes(n_dist,
    n_assign)``, the workspaces of its two launches.  Requests are taken whole,
    in arrival order: a request that does not fit ends the batch, so no later
    request overtakes it."""
    batch, pairs, rb, nd, na = [], 0, 0, 0, 0
    for r in waiting:
        np_ = r.n_pairs(k)
        nd2, na2 = nd + (r.kind == DIST), na + (r.kind == ASSIGN)
        rb2 = rb + req_bytes(r)
        if pairs + np_ > max_pairs or rb2 + ws_bytes(nd2, na2) > budget:
            break
        batch.append(r)
        pairs, rb, nd, na = pairs + np_, rb2, nd2, na2
    return batch


def nearest_centroid(dists) -> int:
    """Index of the smallest cost, as the library's assignment step takes it:
    ties keep the lowest index and NaN never wins (0 when none is finite)."""
    v = np.asarray(dists, np.float64)
    v = np.where(np.isnan(v), np.inf, v)
    return int(np.argmin(v))


def completed(tags, tag: int, starts, open_mask) -> np.ndarray:
    """Requests that are complete: request i owns records [starts[i],
    starts[i + 1]) (``starts`` has one entry more than requests) and is
    complete when each of them carries ``tag``.  Returns the indices of the
    complete requests among those still open (``open_mask``)."""
    posted = np.asarray(tags) == tag
    starts = np.asarray(starts)
    # number of untagged records per request, by a prefix sum over records
    missing = np.concatenate(([0], np.cumsum(~posted)))
    done = (missing[starts[1:]] - missing[starts[:-1]]) == 0
    return np.nonzero(done & open_mask)[0]


def latency_summary(latencies) -> dict:
    """p50 / p99 / max of a list of latencies in seconds, in milliseconds
    (nearest-rank percentiles)."""
    x = np.sort(np.asarray(latencies, np.float64))
    if x.size == 0:
        return {"p50_ms": None, "p99_ms": None, "max_ms": None, "n": 0}

    def rank(q):
        return float(x[min(x.size - 1, max(0, int(np.ceil(q * x.size)) - 1))] * 1e3)

    return {"p50_ms": rank(0.50), "p99_ms": rank(0.99), "max_ms": float(x[-1] * 1e3), "n": int(x.size)}


@dataclass
class _Launch:
    reqs: list
    event: torch.cuda.Event
    done: torch.Tensor    # pinned completion records, one per pair
    tag: int
    starts: np.ndarray    # request i owns pairs [starts[i], starts[i + 1])
    open: np.ndarray      # requests without results yet
    keep: list            # tensors that must outlive the launch
    nbytes: int


@dataclass
class _Grid:
    ctx: Context
    centroids: torch.Tensor | None
    waiting: deque = field(default_factory=deque)
    ws_cache: dict = field(default_factory=dict)


class Server:
    """Continuous-batching server over the library's distance and assignment
    calls.

    ``centroids`` maps a grid size d to a float32 [k, d, d] device tensor of
    centroid histograms (k the same for every grid); grids without centroids
    serve distance requests only.  ``slots`` launches (one per slot, all
    grids together) may be in flight, each of at most ``max_pairs`` pairs; ``mem_budget`` caps the device
    bytes (histograms, workspaces, outputs) of all launches in flight.
    """

    def __init__(self, grids, gamma: float, centroids=None, slots: int = 4, max_pairs: int = 512,
                 mem_budget: int = 8 << 30, tol: float = 1e-3, max_iter: int = 5000,
                 precision="bf16", switch_tol: float = 0.8e-3, device=None, clock=time.perf_counter,
                 kernels=None):
        if slots < 1 or max_pairs < 1 or mem_budget < 1:
            raise ValueError("slots, max_pairs and mem_budget must be positive")
        if not grids:
            raise ValueError("at least one grid is needed")
        centroids = centroids or {}
        ks = {int(c.shape[0]) for c in centroids.values()}
        if len(ks) > 1:
            raise ValueError("every grid needs the same number of centroids")
        self.k = ks.pop() if ks else 0
        if self.k > max_pairs:
            raise ValueError("max_pairs must hold one assignment request (k pairs)")
        self.max_pairs = int(max_pairs)
        self.mem_budget = int(mem_budget)
        self.clock = clock
        self.grids = {}
        kernels = kernels or {}
        for d in grids:
            # distance-kernel tiling: the caller's, else what autotune.tune_kernel
            # chose for this grid and precision in this process, else the default
            kern = kernels.get(d, autotune.choose_kernel(int(d), precision))
            ctx = Context(int(d), gamma, tol=tol, max_iter=max_iter, precision=precision, switch_tol=switch_tol,
                          device=device, kernel=kern)
            cen = centroids.get(d)
            if cen is not None and (cen.dtype != torch.float32 or tuple(cen.shape[1:]) != (d, d)
                                    or cen.device != ctx.device or not cen.is_contiguous()):
                raise ValueError(f"centroids for d={d} must be a contiguous float32 [k, {d}, {d}] on {ctx.device}")
            self.grids[int(d)] = _Grid(ctx, cen)
        dev = next(iter(self.grids.values())).ctx.device
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(slots)]
        self.busy = [None] * slots      # per slot: (grid, launch) in flight, or None
        self.in_flight_bytes = 0
        self.peak_bytes = 0      # most device bytes ever in flight at once
        self.n_launches = 0
        self.done = []
        self._next_id = 0
        self._tag = 0

    def close(self):
        for s in self.streams:
            s.synchronize()
        for g in self.grids.values():
            g.ctx.close()

    # -- submission -------------------------------------------------------
    def submit(self, req: Request, t_arrival: float | None = None) -> Request:
        g = self.grids.get(req.d)
        if g is None:
            raise ValueError(f"no grid d={req.d}")
        if req.kind == ASSIGN and g.centroids is None:
            raise ValueError(f"no centroids at d={req.d}")
        if len(req.diagrams) != (2 if req.kind == DIST else 1):
            raise ValueError("a distance needs two diagrams, an assignment one")
        req.diagrams = [_checked_points(x) for x in req.diagrams]
        if self._launch_bytes(g, [req]) > self.mem_budget:
            # it could never be admitted, and at the head of its queue it would block the grid
            raise ValueError(f"request needs {self._launch_bytes(g, [req])} device bytes, more than the "
                             f"memory budget of {self.mem_budget}")
        req.t_arrival = self.clock() if t_arrival is None else t_arrival
        req.rid = self._next_id
        self._next_id += 1
        g.waiting.append(req)
        return req

    @property
    def pending(self) -> int:
        """Requests without results: waiting, or in a launch that has not
        posted all of their pairs yet."""
        return sum(len(g.waiting) for g in self.grids.values()) + sum(
            int(b[1].open.sum()) for b in self.busy if b is not None)

    @property
    def launches_in_flight(self) -> int:
        return sum(b is not None for b in self.busy)

    # -- memory accounting --------------------------------------------------
    def _req_bytes(self, g: _Grid, r: Request) -> int:
        """Device bytes of one request apart from workspaces: histograms and
        masses of its diagrams, its points and offsets, its outputs."""
        d = g.ctx.d
        nd = len(r.diagrams)
        b = nd * (d * d * 4 + 8 + 8) + sum(len(x) for x in r.diagrams) * 8
        # per pair: indices, outputs (cost, iterations, error, status)
        return b + r.n_pairs(self.k) * (4 + 4 + 8 + 8 + 4 + 4)

    def _ws_bytes(self, g: _Grid, n_dist: int, n_asg: int) -> int:
        """Bytes of a launch with ``n_dist`` distance and ``n_asg`` assignment
        requests beyond its requests' own: the workspace of its one distance
        call (memoised per grid) and, with assignments, the copy of the grid's
        centroids behind the batch's histograms."""
        n = n_dist + n_asg * self.k
        if n == 0:
            return 0
        if n not in g.ws_cache:
            g.ws_cache[n] = g.ctx.workspace_bytes(_lib.PDSINK_OP_DIST, n)
        cen = self.k * g.ctx.d * g.ctx.d * 4 if n_asg else 0
        return g.ws_cache[n] + 64 + cen

    def _launch_bytes(self, g: _Grid, reqs) -> int:
        n_dist = sum(1 for r in reqs if r.kind == DIST)
        return sum(self._req_bytes(g, r) for r in reqs) + self._ws_bytes(g, n_dist, len(reqs) - n_dist)

    # -- the loop -----------------------------------------------------------
    def poll(self) -> int:
        """One turn: retire finished launches, then admit and launch.  Returns
        the number of requests completed in this turn."""
        n = self._retire()
        for s in range(len(self.streams)):
            if self.busy[s] is not None:
                continue
            ready = [g for g in self.grids.values() if g.waiting]
            if not ready:
                break
            g = min(ready, key=lambda e: e.waiting[0].t_arrival)
            budget = self.mem_budget - self.in_flight_bytes
            batch = plan_batch(g.waiting, self.k, self.max_pairs, budget,
                               lambda r, g=g: self._req_bytes(g, r),
                               lambda nd, na, g=g: self._ws_bytes(g, nd, na))
            if not batch:
                if self.in_flight_bytes == 0:
                    raise MemoryError(f"request {g.waiting[0].rid} needs more than the memory budget")
                break
            for _ in batch:
                g.waiting.popleft()
            try:
                L = self._launch(g, self.streams[s], batch)
            except Exception:
                g.waiting.extendleft(reversed(batch))     # back at the head, in order
                raise
            self.busy[s] = (g, L)
            self.in_flight_bytes += L.nbytes
            self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
            self.n_launches += 1
        return n

    def drain(self, timeout_s: float = 60.0):
        """Poll until nothing waits or runs (raises TimeoutError after
        ``timeout_s``)."""
        t0 = time.perf_counter()
        while self.pending or self.launches_in_flight:
            if self.poll() == 0:
                time.sleep(2e-5)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{self.pending} requests still pending")

    def _retire(self) -> int:
        """Results of the requests whose pairs have all posted; release of the
        launches that have ended."""
        n = 0
        for s, b in enumerate(self.busy):
            if b is None:
                continue
            L = b[1]
            # query the event before reading the records: once it has passed,
            # every record of the launch is posted and visible
            ended = L.event.query()
            rec = done_view(L.done)
            fin = completed(rec["tag"], L.tag, L.starts, L.open)
            if ended and len(fin) != int(L.open.sum()):
                raise RuntimeError(f"launch ended with {int(L.open.sum()) - len(fin)} requests unposted")
            if len(fin):
                now = self.clock()
                for i in fin:
                    r, lo, hi = L.reqs[i], L.starts[i], L.starts[i + 1]
                    part = rec[lo:hi]
                    if r.kind == DIST:
                        r.cost = float(part["cost"][0])
                    else:
                        r.dists = part["cost"].copy()
                        r.assign = nearest_centroid(r.dists)
                    r.status = part["status"].copy()
                    r.t_done = now
                    self.done.append(r)
                L.open[fin] = False
                n += len(fin)
            if ended:
                self.in_flight_bytes -= L.nbytes
                self.busy[s] = None
        return n

    def _launch(self, g: _Grid, stream, reqs) -> _Launch:
        ctx, dev, k = g.ctx, g.ctx.device, self.k
        keep = []
        nbytes = self._launch_bytes(g, reqs)
        # histograms of the batch's diagrams, in request order, then (with
        # assignments) the centroids; pairs in request order
        n_up = sum(len(r.diagrams) for r in reqs)
        any_asg = any(r.kind == ASSIGN for r in reqs)
        ia, ib, starts, row = [], [], [0], 0
        for r in reqs:
            if r.kind == DIST:
                ia.append(row)
                ib.append(row + 1)
                row += 2
            else:
                ia += [row] * k
                ib += range(n_up, n_up + k)
                row += 1
            starts.append(len(ia))
        n = len(ia)
        self._tag = self._tag % 0xFFFFFFFF + 1
        done = done_records(n)
        with torch.cuda.stream(stream):
            buf = torch.empty((n_up + (k if any_asg else 0), ctx.d, ctx.d), dtype=torch.float32, device=dev)
            _upload(ctx, [x for r in reqs for x in r.diagrams], keep, out=buf)
            if any_asg:
                buf[n_up:].copy_(g.centroids)
            hidx = torch.tensor([ia, ib], dtype=torch.int32).pin_memory()
            didx = hidx.to(dev, non_blocking=True)
            res = sinkhorn_dist_batch_notify(ctx, buf, buf, didx[0], didx[1], done, self._tag,
                                             check_indices=False)
            keep += [buf, hidx, didx, res]
            ev = torch.cuda.Event()
            ev.record(stream)
        return _Launch(reqs, ev, done, self._tag, np.asarray(starts), np.ones(len(reqs), bool), keep, nbytes)


def _checked_points(x) -> np.ndarray:
    """A diagram as float32 [n, 2].  Raises ValueError for a point that the
    discretisation would drop (outside [0, 1]^2, non-finite, or birth >
    death), so that no request is served without part of its diagram."""
    a = np.asarray(x, dtype=np.float32)
    if a.size % 2:
        raise ValueError("a diagram is an array of (birth, death) pairs")
    a = np.ascontiguousarray(a.reshape(-1, 2))
    with np.errstate(invalid="ignore"):
        bad = ~np.isfinite(a).all(axis=1) | (a < 0).any(axis=1) | (a > 1).any(axis=1) | (a[:, 0] > a[:, 1])
    if bad.any():
        raise ValueError(f"{int(bad.sum())} points outside [0, 1]^2, non-finite or with birth > death")
    return a


def _upload(ctx: Context, diagrams, keep, out=None) -> torch.Tensor:
    """Histograms of ``diagrams`` on the current stream (CSR points copied from
    pinned host memory), into the first rows of ``out`` when given."""
    counts = np.array([len(x) for x in diagrams], np.int64)
    off = np.zeros(len(diagrams) + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    pts = np.concatenate([np.asarray(x, np.float32).reshape(-1, 2) for x in diagrams], 0) if off[-1] else \
        np.zeros((0, 2), np.float32)
    hp = torch.from_numpy(np.ascontiguousarray(pts)).pin_memory()
    ho = torch.from_numpy(off).pin_memory()
    dp = hp.to(ctx.device, non_blocking=True)
    do = ho.to(ctx.device, non_blocking=True)
    keep += [hp, ho, dp, do]
    hist, mass, n_bad = pd_discretize(ctx, dp, do, hist=out)
    keep += [mass, n_bad]
    return hist


def run_stream(server: Server, stream, realtime: bool = True, timeout_s: float = 120.0):
    """Feed ``stream`` (dicts with keys ``t``, ``kind``, ``d``, ``diagrams``,
    arrival times in seconds) to ``server``.  With ``realtime`` a request is
    submitted once the clock passes its arrival time and its latency counts
    from that arrival time; otherwise all are submitted at once.  Returns the
    requests (with results) and the wall time from the first arrival to the
    last completion.  Returns once every launch has ended as well."""
    reqs = [Request(s["kind"], s["d"], s["diagrams"]) for s in stream]
    t0 = server.clock()
    i = 0
    while i < len(reqs) or server.pending or server.launches_in_flight:
        now = server.clock()
        while i < len(reqs) and (not realtime or stream[i]["t"] <= now - t0):
            server.submit(reqs[i], t_arrival=t0 + (stream[i]["t"] if realtime else 0.0))
            i += 1
        if server.poll() == 0:
            time.sleep(2e-5)
        if server.clock() - t0 > timeout_s:
            raise TimeoutError(f"{server.pending} requests still pending")
    t_end = max((r.t_done for r in reqs), default=t0)
    return reqs, t_end - t0
