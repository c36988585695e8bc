"""MI355X (gfx950) persistence-diagram Sinkhorn library: Python binding.

Thin marshalling over the C ABI of ``include/pdsink.h`` (loaded with ctypes
from the in-tree ``libpdsink.so``).  Every step of the computation runs in the
library's HIP kernels; PyTorch only provides device memory and the current
stream.  The functions keep the C names:

* ``pd_discretize``       - diagrams (CSR points) to d x d histograms + masses
* ``sinkhorn_dist_batch`` - Algorithm 1 for a batch of pairs
* ``pd_barycenter``       - Algorithm 2
* ``kmeans_assign``       - k-means assignment step
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import PdsinkError  # noqa: F401

__all__ = ["Context", "pd_discretize", "sinkhorn_dist_batch", "sinkhorn_dist_batch_noalloc",
           "sinkhorn_dist_batch_notify", "done_records", "done_view", "pd_barycenter",
           "kmeans_assign", "pd_sharpen", "pd_quantize", "PdsinkError", "FP32", "BF16_REFINE"]

FP32 = _lib.PDSINK_FP32
BF16_REFINE = _lib.PDSINK_BF16_REFINE
_PREC = {"fp32": FP32, "bf16": BF16_REFINE, "bf16_refine": BF16_REFINE, FP32: FP32, BF16_REFINE: BF16_REFINE}
# distance-kernel tiling: "auto" (the default per grid), "resident" (d in 33..100), "general"
_KERNEL = {"auto": _lib.PDSINK_KERNEL_AUTO, "resident": _lib.PDSINK_KERNEL_RESIDENT,
           "general": _lib.PDSINK_KERNEL_GENERAL, 0: 0, 1: 1, 2: 2}


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, name, dtype, dev):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != dev:
        raise ValueError(f"{name} must be on {dev}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """A ``pdsink_ctx``: grid size, ground exponent, gamma and stopping rule."""

    def __init__(self, d: int, gamma: float, p: float = 2.0, tol: float = 1e-3, max_iter: int = 1000,
                 precision="fp32", switch_tol: float = 1.5e-3, device=None, kernel="auto"):
        lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device_index = int(torch.device("cuda", device).index if not isinstance(device, int) else device)
        self.device = torch.device("cuda", self.device_index)
        prm = _lib.Params(int(d), float(p), float(gamma), float(tol), int(max_iter), _PREC[precision],
                          float(switch_tol), _KERNEL[kernel])
        h = ctypes.c_void_p()
        _lib.check("pdsink_ctx_create", lib.pdsink_ctx_create(ctypes.byref(prm), self.device_index, ctypes.byref(h)))
        self._h = h
        self.d, self.gamma, self.p, self.tol, self.max_iter = int(d), float(gamma), float(p), float(tol), int(max_iter)
        self.precision = _PREC[precision]
        self.switch_tol = float(switch_tol)
        self.kernel = _KERNEL[kernel]

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().pdsink_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def workspace_bytes(self, op: int, n_items: int) -> int:
        n = ctypes.c_size_t()
        _lib.check("pdsink_workspace_bytes",
                   _lib.load().pdsink_workspace_bytes(self.handle, op, int(n_items), ctypes.byref(n)))
        return int(n.value)

    def workspace(self, op: int, n_items: int) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(op, n_items), 1), dtype=torch.uint8, device=self.device)


def pd_discretize(ctx: Context, pts: torch.Tensor, offsets: torch.Tensor, hist=None, mass=None, n_bad=None):
    """Histograms [n, d, d] (float32) and masses [n] (float64) of CSR diagrams.

    Returns ``(hist, mass, n_bad)``; ``n_bad`` is a device int32 [1] counter of
    rejected points (added to when given)."""
    dev = ctx.device
    _need(pts, "pts", torch.float32, dev)
    _need(offsets, "offsets", torch.int64, dev)
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs at least one entry")
    d = ctx.d
    hist = torch.empty((n, d, d), dtype=torch.float32, device=dev) if hist is None else hist
    mass = torch.empty((n,), dtype=torch.float64, device=dev) if mass is None else mass
    n_bad = torch.zeros((1,), dtype=torch.int32, device=dev) if n_bad is None else n_bad
    _need(hist, "hist", torch.float32, dev)
    _need(mass, "mass", torch.float64, dev)
    _need(n_bad, "n_bad", torch.int32, dev)
    if hist.numel() < n * d * d or mass.numel() < n:
        raise ValueError("output too small")
    _lib.check("pd_discretize", _lib.load().pd_discretize(ctx.handle, _vp(pts), _vp(offsets), n, _vp(hist),
                                                          _vp(mass), _vp(n_bad), _stream()))
    return hist, mass, n_bad


@dataclass
class DistResult:
    cost: torch.Tensor      # float64 [n]
    iters: torch.Tensor     # int32 [n, 2]: BF16 iterations, FP32 iterations
    err: torch.Tensor       # float32 [n]
    status: torch.Tensor    # int32 [n]
    upper: torch.Tensor | None = None   # float64 [n]: <R_t, C> of the rounded plan (bounds=True)
    lower: torch.Tensor | None = None   # float64 [n]: c-transform dual bound (bounds=True)


def _pair_args(ctx, hist_a, hist_b, ia, ib, out, check_indices):
    dev = ctx.device
    for t, nm in ((hist_a, "hist_a"), (hist_b, "hist_b")):
        _need(t, nm, torch.float32, dev)
        if t.dim() != 3 or t.shape[1:] != (ctx.d, ctx.d):
            raise ValueError(f"{nm} must be [n, {ctx.d}, {ctx.d}]")
    _need(ia, "ia", torch.int32, dev)
    _need(ib, "ib", torch.int32, dev)
    n = ia.numel()
    if ib.numel() != n:
        raise ValueError("ia and ib differ in length")
    if n and check_indices and (int(ia.min()) < 0 or int(ia.max()) >= hist_a.shape[0]
              or int(ib.min()) < 0 or int(ib.max()) >= hist_b.shape[0]):
        raise IndexError("pair index out of range")
    if out is None:
        out = DistResult(torch.empty(n, dtype=torch.float64, device=dev),
                         torch.empty((n, 2), dtype=torch.int32, device=dev),
                         torch.empty(n, dtype=torch.float32, device=dev),
                         torch.empty(n, dtype=torch.int32, device=dev))
    return n, out


def sinkhorn_dist_batch(ctx: Context, hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor,
                        ib: torch.Tensor, out: DistResult | None = None, ws: torch.Tensor | None = None,
                        check_indices: bool = True, bounds: bool = False,
                        state: torch.Tensor | None = None) -> DistResult:
    """Algorithm 1 on pairs (hist_a[ia[q]], hist_b[ib[q]]).

    ``bounds`` also returns the error-control bounds of section 3 in
    ``upper`` and ``lower`` (lower <= exact transport value <= upper).

    ``state`` (float64 [n, d*d + 1]: natural log of v on the grid cells, then
    the diagonal bin) is Algorithm 1's initial v, overwritten with log v at
    stopping; None starts from v = 1.  Not combined with ``bounds``.

    ``check_indices`` reads the index ranges back to the host (a stream
    synchronisation); pass False inside graph capture, where the caller
    guarantees that every index addresses its pool."""
    dev = ctx.device
    n, out = _pair_args(ctx, hist_a, hist_b, ia, ib, out, check_indices)
    if state is not None:
        if bounds:
            raise ValueError("state and bounds are not combined")
        _need(state, "state", torch.float64, dev)
        if state.shape != (n, ctx.d * ctx.d + 1):
            raise ValueError(f"state must be [{n}, {ctx.d * ctx.d + 1}]")
    if ws is None:
        ws = ctx.workspace(_lib.PDSINK_OP_DIST if state is None else _lib.PDSINK_OP_DIST_WARM, n)
    if bounds:
        if out.upper is None:
            out.upper = torch.empty(n, dtype=torch.float64, device=dev)
        if out.lower is None:
            out.lower = torch.empty(n, dtype=torch.float64, device=dev)
        _lib.check("sinkhorn_dist_bounds_batch", _lib.load().sinkhorn_dist_bounds_batch(
            ctx.handle, n, _vp(hist_a), _vp(hist_b), _vp(ia), _vp(ib), _vp(out.cost), _vp(out.iters),
            _vp(out.err), _vp(out.status), _vp(out.upper), _vp(out.lower), _vp(ws), ws.numel(), _stream()))
        return out
    _lib.check("sinkhorn_dist_batch", _lib.load().sinkhorn_dist_batch(
        ctx.handle, n, _vp(hist_a), _vp(hist_b), _vp(ia), _vp(ib), _vp(state), _vp(out.cost), _vp(out.iters),
        _vp(out.err), _vp(out.status), _vp(ws), ws.numel(), _stream()))
    return out


def done_records(n: int) -> torch.Tensor:
    """Pinned host memory for ``n`` completion records (``pdsink_done``), all
    tags zero; view it with ``done_view``."""
    return torch.zeros(n * _lib.DONE_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)


def done_view(done: torch.Tensor) -> np.ndarray:
    """The records of ``done`` (from ``done_records``) as a numpy structured
    array over the same host memory (fields cost, err, status, iters, tag)."""
    return done.numpy().view(_lib.DONE_DTYPE)


def sinkhorn_dist_batch_notify(ctx: Context, hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor,
                               ib: torch.Tensor, done: torch.Tensor, tag: int, out: DistResult | None = None,
                               ws: torch.Tensor | None = None, check_indices: bool = True) -> DistResult:
    """``sinkhorn_dist_batch`` that posts each pair's outputs to the pinned
    records ``done`` (``done_records(n)``) as soon as they are final, with
    ``tag`` (non-zero, new per call on reused records) stored last."""
    n, out = _pair_args(ctx, hist_a, hist_b, ia, ib, out, check_indices)
    if not isinstance(done, torch.Tensor) or done.device.type != "cpu" or done.dtype != torch.uint8 \
            or not done.is_contiguous() or not done.is_pinned():
        raise ValueError("done must be pinned contiguous uint8 host memory (done_records)")
    if done.numel() < n * _lib.DONE_DTYPE.itemsize:
        raise ValueError("done holds fewer records than pairs")
    if not 0 < int(tag) < 1 << 32:
        raise ValueError("tag must be a non-zero uint32")
    if ws is None:
        ws = ctx.workspace(_lib.PDSINK_OP_DIST, n)
    _lib.check("sinkhorn_dist_batch_notify", _lib.load().sinkhorn_dist_batch_notify(
        ctx.handle, n, _vp(hist_a), _vp(hist_b), _vp(ia), _vp(ib), _vp(out.cost), _vp(out.iters),
        _vp(out.err), _vp(out.status), ctypes.c_void_p(done.data_ptr()), int(tag), _vp(ws), ws.numel(),
        _stream()))
    return out


def sinkhorn_dist_batch_noalloc(ctx: Context, hist_a: torch.Tensor, hist_b: torch.Tensor, ia: torch.Tensor,
                                ib: torch.Tensor, out: DistResult | None = None,
                                check_indices: bool = True) -> DistResult:
    """``sinkhorn_dist_batch`` on the library's static scratch array: the call
    allocates no device memory (pass ``out`` to allocate nothing here either).
    At most ``PDSINK_NOALLOC_MAX_PAIRS`` pairs; calls that overlap on one GPU race."""
    n, out = _pair_args(ctx, hist_a, hist_b, ia, ib, out, check_indices)
    _lib.check("sinkhorn_dist_batch_noalloc", _lib.load().sinkhorn_dist_batch_noalloc(
        ctx.handle, n, _vp(hist_a), _vp(hist_b), _vp(ia), _vp(ib), _vp(out.cost), _vp(out.iters),
        _vp(out.err), _vp(out.status), _stream()))
    return out


def pd_sharpen(ctx: Context, z: torch.Tensor, h0: float, beta: torch.Tensor | None = None) -> torch.Tensor:
    """Entropic sharpening of histograms ``z`` ([n, d, d] or [d, d] float32, in
    place) to entropy ``h0`` (nats).  Returns the exponents used (float64 [n];
    1 = unchanged, inf = the even split over the maximal cells)."""
    dev = ctx.device
    _need(z, "z", torch.float32, dev)
    zz = z if z.dim() == 3 else z.unsqueeze(0)
    if zz.dim() != 3 or zz.shape[1:] != (ctx.d, ctx.d):
        raise ValueError(f"z must be [n, {ctx.d}, {ctx.d}] or [{ctx.d}, {ctx.d}]")
    n = zz.shape[0]
    if beta is None:
        beta = torch.empty(n, dtype=torch.float64, device=dev)
    _need(beta, "beta", torch.float64, dev)
    if beta.numel() != n:
        raise ValueError("beta needs one entry per histogram")
    _lib.check("pd_sharpen", _lib.load().pd_sharpen(ctx.handle, n, _vp(zz), float(h0), _vp(beta), _stream()))
    return beta


def pd_quantize(ctx: Context, z: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Histograms ``z`` ([n, d, d] or [d, d] float32) rounded cell by cell to
    point counts (float32 integers); ``out`` may be ``z`` itself."""
    dev = ctx.device
    _need(z, "z", torch.float32, dev)
    if z.shape[-2:] != (ctx.d, ctx.d) or z.dim() not in (2, 3):
        raise ValueError(f"z must be [n, {ctx.d}, {ctx.d}] or [{ctx.d}, {ctx.d}]")
    if out is None:
        out = torch.empty_like(z)
    _need(out, "out", torch.float32, dev)
    if out.shape != z.shape:
        raise ValueError("out must have the shape of z")
    n = 1 if z.dim() == 2 else z.shape[0]
    _lib.check("pd_quantize", _lib.load().pd_quantize(ctx.handle, n, _vp(z), _vp(out), _stream()))
    return out


def kmeans_assign(ctx: Context, hist: torch.Tensor, centroids: torch.Tensor, ws: torch.Tensor | None = None):
    """Assignment step: returns ``(assign int32 [n], dist float64 [n, k], status int32 [n, k])``."""
    dev = ctx.device
    _need(hist, "hist", torch.float32, dev)
    _need(centroids, "centroids", torch.float32, dev)
    n, k = hist.shape[0], centroids.shape[0]
    assign = torch.empty(n, dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.float64, device=dev)
    status = torch.empty((n, k), dtype=torch.int32, device=dev)
    if ws is None:
        ws = ctx.workspace(_lib.PDSINK_OP_KMEANS, n * k)
    _lib.check("kmeans_assign", _lib.load().kmeans_assign(
        ctx.handle, n, _vp(hist), k, _vp(centroids), _vp(assign), _vp(dist), _vp(status), _vp(ws), ws.numel(),
        _stream()))
    return assign, dist, status


def pd_barycenter(ctx: Context, hist: torch.Tensor, lam: float = 5.0, max_outer: int = 50,
                  energy_rtol: float = 0.01, z: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Algorithm 2: returns ``(z [d, d] float32, energy float, outer steps int)``."""
    dev = ctx.device
    _need(hist, "hist", torch.float32, dev)
    n = hist.shape[0]
    init = z is None
    if z is None:
        z = torch.empty((ctx.d, ctx.d), dtype=torch.float32, device=dev)
    _need(z, "z", torch.float32, dev)
    if ws is None:
        ws = ctx.workspace(_lib.PDSINK_OP_BARYCENTER, n)
    energy = ctypes.c_double()
    outer = ctypes.c_int32()
    _lib.check("pd_barycenter", _lib.load().pd_barycenter(
        ctx.handle, n, _vp(hist), float(lam), int(max_outer), float(energy_rtol), int(init), _vp(z),
        ctypes.byref(energy), ctypes.byref(outer), _vp(ws), ws.numel(), _stream()))
    return z, float(energy.value), int(outer.value)


def kmeans_lloyd(ctx: Context, hist: torch.Tensor, k: int, rounds: int, init, lam: float = 5.0,
                 max_outer: int = 10, energy_rtol: float = 0.01):
    """k-means by Lloyd rounds (section 5).  ``init``: k distinct diagram
    indices of the initial centroids (a seeded draw made by the caller).
    Returns ``(centroids [k, d, d], assign [n], objective [rounds] numpy)``."""
    dev = ctx.device
    _need(hist, "hist", torch.float32, dev)
    n = hist.shape[0]
    init = np.ascontiguousarray(np.asarray(init, dtype=np.int32))
    if init.shape != (k,):
        raise ValueError("init must hold k indices")
    cents = torch.empty((k, ctx.d, ctx.d), dtype=torch.float32, device=dev)
    assign = torch.empty((n,), dtype=torch.int32, device=dev)
    obj = np.zeros(max(rounds, 1), dtype=np.float64)
    nb = ctypes.c_size_t()
    lib = _lib.load()
    _lib.check("pdsink_lloyd_workspace_bytes", lib.pdsink_lloyd_workspace_bytes(ctx.handle, n, k, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
    _lib.check("kmeans_lloyd", lib.kmeans_lloyd(
        ctx.handle, n, _vp(hist), int(k), init.ctypes.data_as(ctypes.c_void_p), int(rounds), float(lam),
        int(max_outer), float(energy_rtol), _vp(cents), _vp(assign), obj.ctypes.data_as(ctypes.c_void_p), _vp(ws),
        ws.numel(), _stream()))
    return cents, assign, obj[:rounds]
