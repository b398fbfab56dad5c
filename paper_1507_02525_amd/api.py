"""PyTorch-facing wrappers of the C ABI.

PyTorch supplies device memory and the current stream; every step of the
transform runs in libmrdft.so.  Names follow the C ABI (``mrdft_forward`` ...)
with thin tensor helpers on top:

* :class:`Plan` owns an ``mrdft_plan_t`` (uniform or ragged batch).
* :func:`forward` / :func:`adjoint` take and return tensors.
* :class:`MrDFT` is a ``torch.autograd.Function``; its backward is the adjoint
  kernel (the transform is linear, so nothing is saved).
* :func:`spectral_loss` is the multi-resolution spectral loss with a
  hand-written backward that recomputes the level spectra.
"""
from __future__ import annotations

import collections
import ctypes
import threading

import numpy as np
import torch

from . import _binding as B


def _stream_ptr(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owner of one ``mrdft_plan_t``.

    Uniform batch: ``Plan(m=m, batch=B, dtype="c64"|"r32")``.
    Ragged batch:  ``Plan(offsets=int64 array [batch+1], dtype=...)``.
    ``tune=True`` times the candidate schedules at creation; ``graph=True``
    replays mrdft_forward from a captured HIP graph; ``levels=(lo, hi)`` keeps
    only those levels (compact output, see mrdft_plan_create_levels);
    ``half=True`` (real input) stores each window as its packed half spectrum
    (L/2 values, value 0 = (Y[0], Y[L/2]); see MRDFT_FLAG_HALF).
    """

    def __init__(self, m: int = 0, batch: int = 1, offsets=None, dtype: str = "c64", device=None,
                 tune: bool = False, graph: bool = False, levels=None, half: bool = False):
        lib = B.lib()
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        code = {"c64": B.MRDFT_C64, "r32": B.MRDFT_R32}.get(dtype)
        if code is None:
            raise ValueError("dtype must be 'c64' or 'r32'")
        h = ctypes.c_void_p()
        off_arr = None
        if offsets is not None:
            off_arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
            batch = len(off_arr) - 1
            offp = off_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        else:
            offp = None
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            flags = (B.MRDFT_FLAG_TUNE if tune else 0) | (B.MRDFT_FLAG_GRAPH if graph else 0) \
                | (B.MRDFT_FLAG_HALF if half else 0)
            lo, hi = (1, B.MRDFT_MAX_ORDER) if levels is None else (int(levels[0]), int(levels[1]))
            B.check(lib.mrdft_plan_create_levels(ctypes.byref(h), int(m), int(batch), offp, code, flags, lo, hi,
                                                 stream))
        self.levels = (lo, hi)
        self.half = bool(half)
        self.handle = h
        self.m = int(m)
        self.batch = int(batch)
        self.ragged = offsets is not None
        n_in = ctypes.c_int64()
        n_out = ctypes.c_int64()
        B.check(lib.mrdft_plan_sizes(h, ctypes.byref(n_in), ctypes.byref(n_out)))
        self.n_in = n_in.value
        self.n_out = n_out.value

    # -- C ABI mirrors -------------------------------------------------------
    def schedule(self) -> dict:
        """Forward schedule chosen at creation: tile_log, grid, order, serial."""
        t, g, o = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        B.check(B.lib().mrdft_plan_schedule(self.handle, ctypes.byref(t), ctypes.byref(g), ctypes.byref(o)))
        return {"tile_log": t.value, "grid": g.value, "order": B.ORDERS[o.value & 0xff],
                "serial": bool(o.value & B.MRDFT_SCHED_SERIAL), "after": bool(o.value & B.MRDFT_SCHED_AFTER)}

    def set_schedule(self, tile_log: int, grid: int, order: str, serial: bool = False, after: bool = False):
        """Pin the forward schedule (values as returned by schedule())."""
        code = B.ORDERS.index(order) | (B.MRDFT_SCHED_SERIAL if serial else 0) | (B.MRDFT_SCHED_AFTER if after else 0)
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            B.check(B.lib().mrdft_plan_set_schedule(self.handle, int(tile_log), int(grid), code, stream))

    def output_offsets(self) -> np.ndarray:
        out = np.empty(self.batch + 1, dtype=np.int64)
        B.check(B.lib().mrdft_plan_output_offsets(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def _check_in(self, x: torch.Tensor, what: str):
        want = torch.complex64 if self.dtype == "c64" else torch.float32
        if x.dtype != want:
            raise TypeError("%s must be %s, got %s" % (what, want, x.dtype))
        if x.device != self.device or not x.is_contiguous() or x.numel() != self.n_in:
            raise ValueError("%s must be a contiguous %s tensor of %d elements on %s"
                             % (what, want, self.n_in, self.device))

    def _check_out(self, Y: torch.Tensor, what: str):
        if Y.dtype != torch.complex64 or Y.device != self.device or not Y.is_contiguous() \
                or Y.numel() != self.n_out:
            raise ValueError("%s must be a contiguous complex64 tensor of %d elements on %s"
                             % (what, self.n_out, self.device))

    def mrdft_forward(self, x: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
        self._check_in(x, "x")
        self._check_out(Y, "Y")
        B.check(B.lib().mrdft_forward(self.handle, _ptr(x), _ptr(Y), _stream_ptr(x)))
        return Y

    def mrdft_adjoint(self, gY: torch.Tensor, gx: torch.Tensor) -> torch.Tensor:
        self._check_out(gY, "gY")
        self._check_in(gx, "gx")
        B.check(B.lib().mrdft_adjoint(self.handle, _ptr(gY), _ptr(gx), _stream_ptr(gY)))
        return gx

    def _check_buf(self, t: torch.Tensor, dtype, numel: int, what: str):
        if t.dtype != dtype or t.device != self.device or not t.is_contiguous() or t.numel() != numel:
            raise ValueError("%s must be a contiguous %s tensor of %d elements on %s" % (what, dtype, numel, self.device))

    def _check_loss(self, x, z, num_den):
        if self.dtype != "r32" or self.ragged:
            raise ValueError("the spectral loss needs a uniform real (r32) plan")
        self._check_in(x, "x")
        self._check_in(z, "z")
        self._check_buf(num_den, torch.float64, self.batch * self.m * 2, "num_den")

    def mrdft_spectral_loss_fwd(self, x, z, num_den, L):
        self._check_loss(x, z, num_den)
        self._check_buf(L, torch.float32, 1, "L")
        B.check(B.lib().mrdft_spectral_loss_fwd(self.handle, _ptr(x), _ptr(z), _ptr(num_den), _ptr(L),
                                                _stream_ptr(x)))
        return num_den, L

    def mrdft_spectral_loss_bwd(self, x, z, num_den, gL, gx):
        self._check_loss(x, z, num_den)
        self._check_buf(gL, torch.float32, 1, "gL")
        self._check_in(gx, "gx")
        B.check(B.lib().mrdft_spectral_loss_bwd(self.handle, _ptr(x), _ptr(z), _ptr(num_den), _ptr(gL), _ptr(gx),
                                                _stream_ptr(x)))
        return gx

    def set_profiling(self, enable: bool):
        B.check(B.lib().mrdft_plan_set_profiling(self.handle, 1 if enable else 0))

    def read_profile(self) -> dict:
        """{kind: (total_ms, launches)} since the last read (waits for the events)."""
        n = len(B.KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        B.check(B.lib().mrdft_plan_read_profile(self.handle, n, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(B.KERNEL_KINDS)}

    # -- tensor helpers --------------------------------------------------------
    def forward(self, x: torch.Tensor) -> torch.Tensor:
        Y = torch.empty(self.n_out, dtype=torch.complex64, device=self.device)
        self.mrdft_forward(x.contiguous(), Y)
        if not self.ragged:
            kept = min(self.levels[1], self.m) - self.levels[0] + 1
            Y = Y.view(self.batch, kept, (1 << self.m) >> (1 if self.half else 0))
        return Y

    def adjoint(self, gY: torch.Tensor) -> torch.Tensor:
        want = torch.complex64 if self.dtype == "c64" else torch.float32
        gx = torch.empty(self.n_in, dtype=want, device=self.device)
        self.mrdft_adjoint(gY.contiguous().view(-1), gx)
        if not self.ragged:
            gx = gx.view(self.batch, 1 << self.m)
        return gx

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            B.check(B.lib().mrdft_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan2D:
    """Owner of one ``mrdft_plan2d_t``: the separable 2-D transform of
    ``batch`` images of 2^m1 x 2^m2 samples (see mrdft_plan2d_create).
    ``forward`` returns complex64 of shape (batch, m1, N1, m2, N2): the plane
    of the level pair (i1, i2) is ``Y[:, i1-1, :, i2-1, :]``."""

    def __init__(self, m1: int, m2: int, batch: int = 1, dtype: str = "c64", device=None):
        lib = B.lib()
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        code = {"c64": B.MRDFT_C64, "r32": B.MRDFT_R32}.get(dtype)
        if code is None:
            raise ValueError("dtype must be 'c64' or 'r32'")
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            B.check(lib.mrdft_plan2d_create(ctypes.byref(h), int(m1), int(m2), int(batch), code, stream))
        self.handle = h
        self.m1, self.m2, self.batch = int(m1), int(m2), int(batch)
        n_in = ctypes.c_int64()
        n_out = ctypes.c_int64()
        B.check(lib.mrdft_plan2d_sizes(h, ctypes.byref(n_in), ctypes.byref(n_out)))
        self.n_in, self.n_out = n_in.value, n_out.value

    def _want(self):
        return torch.complex64 if self.dtype == "c64" else torch.float32

    def mrdft_forward2d(self, x: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
        if x.dtype != self._want() or not x.is_contiguous() or x.numel() != self.n_in or x.device != self.device:
            raise ValueError("x must be a contiguous %s tensor of %d elements on %s"
                             % (self._want(), self.n_in, self.device))
        if Y.dtype != torch.complex64 or not Y.is_contiguous() or Y.numel() != self.n_out or Y.device != self.device:
            raise ValueError("Y must be a contiguous complex64 tensor of %d elements" % self.n_out)
        B.check(B.lib().mrdft_forward2d(self.handle, _ptr(x), _ptr(Y), _stream_ptr(x)))
        return Y

    def mrdft_adjoint2d(self, gY: torch.Tensor, gx: torch.Tensor) -> torch.Tensor:
        if gY.dtype != torch.complex64 or not gY.is_contiguous() or gY.numel() != self.n_out \
                or gY.device != self.device:
            raise ValueError("gY must be a contiguous complex64 tensor of %d elements on %s" % (self.n_out, self.device))
        if gx.dtype != self._want() or not gx.is_contiguous() or gx.numel() != self.n_in or gx.device != self.device:
            raise ValueError("gx must be a contiguous %s tensor of %d elements on %s"
                             % (self._want(), self.n_in, self.device))
        B.check(B.lib().mrdft_adjoint2d(self.handle, _ptr(gY), _ptr(gx), _stream_ptr(gY)))
        return gx

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        Y = torch.empty(self.n_out, dtype=torch.complex64, device=self.device)
        self.mrdft_forward2d(x.contiguous(), Y)
        return Y.view(self.batch, self.m1, 1 << self.m1, self.m2, 1 << self.m2)

    def adjoint(self, gY: torch.Tensor) -> torch.Tensor:
        gx = torch.empty(self.n_in, dtype=self._want(), device=self.device)
        self.mrdft_adjoint2d(gY.contiguous().view(-1), gx)
        return gx.view(self.batch, 1 << self.m1, 1 << self.m2)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            B.check(B.lib().mrdft_plan2d_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Plans of the tensor helpers, least recently used first.  A plan's workspace
# (pass scratch, adjoint scratch, loss buffers) is single, so two calls on one
# plan must not overlap: the key holds the stream the call is queued on (calls
# on one stream run in order) and the calling thread (a plan's host state is
# not shared between threads).  At most CACHE_SIZE plans are kept; an evicted
# plan is destroyed when its last user (e.g. an autograd context) drops it,
# and destruction waits for its queued work.
CACHE_SIZE = 8
_cache: "collections.OrderedDict" = collections.OrderedDict()
_cache_lock = threading.Lock()


def get_plan(m: int, batch: int, dtype: str, device) -> Plan:
    device = torch.device(device)
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (int(m), int(batch), dtype, str(device), int(stream), threading.get_ident())
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(m=m, batch=batch, dtype=dtype, device=device)
            _cache[key] = p
        _cache.move_to_end(key)
        while len(_cache) > CACHE_SIZE:
            _cache.popitem(last=False)
        return p


def clear_plan_cache():
    """Drop every cached plan (each is destroyed once no caller holds it)."""
    with _cache_lock:
        _cache.clear()


def _order_of(n: int) -> int:
    m = int(n).bit_length() - 1
    if n < 2 or (1 << m) != n:
        raise ValueError("signal length must be 2^m with m >= 1, got %d" % n)
    return m


def _dtype_name(x: torch.Tensor) -> str:
    if x.dtype == torch.complex64:
        return "c64"
    if x.dtype == torch.float32:
        return "r32"
    raise TypeError("x must be complex64 or float32, got %s" % x.dtype)


def forward(x: torch.Tensor) -> torch.Tensor:
    """x (..., N) complex64 or float32 on a GPU -> (..., m, N) complex64."""
    if not x.is_cuda:
        raise ValueError("x must be a GPU tensor (there is no CPU path)")
    lead = x.shape[:-1]
    m = _order_of(x.shape[-1])
    xb = x.reshape(-1, x.shape[-1]).contiguous()
    p = get_plan(m, xb.shape[0], _dtype_name(x), x.device)
    return p.forward(xb).reshape(*lead, m, x.shape[-1])


def adjoint(gY: torch.Tensor, real: bool = False) -> torch.Tensor:
    """gY (..., m, N) complex64 -> gx (..., N) (float32 real part if real=True)."""
    m = gY.shape[-2]
    n = gY.shape[-1]
    if _order_of(n) != m:
        raise ValueError("gY must have shape (..., m, 2^m)")
    lead = gY.shape[:-2]
    g = gY.reshape(-1, m, n).contiguous()
    p = get_plan(m, g.shape[0], "r32" if real else "c64", gY.device)
    return p.adjoint(g).reshape(*lead, n)


class MrDFT(torch.autograd.Function):
    """Y = MrDFT(x); backward is the adjoint kernel (real part for real x)."""

    @staticmethod
    def forward(ctx, x):
        ctx.real = x.dtype == torch.float32
        return forward(x)

    @staticmethod
    def backward(ctx, gY):
        return adjoint(gY.to(torch.complex64), real=ctx.real)


def mrdft(x: torch.Tensor) -> torch.Tensor:
    return MrDFT.apply(x)


def _check_loss_inputs(x: torch.Tensor, z: torch.Tensor):
    if x.dtype != torch.float32 or z.dtype != torch.float32:
        raise TypeError("spectral_loss takes float32 x and z")
    if x.shape != z.shape or x.dim() == 0:
        raise ValueError("x and z must have one shape (..., N), got %s and %s" % (tuple(x.shape), tuple(z.shape)))
    if not x.is_cuda or x.device != z.device:
        raise ValueError("x and z must be on one GPU (there is no CPU path)")


class SpectralLoss(torch.autograd.Function):
    """L = sum_b (1/m) sum_i ||Y^(i)(x_b) - Y^(i)(z_b)||^2 / ||Y^(i)(z_b)||^2 (z not differentiated)."""

    @staticmethod
    def forward(ctx, x, z):
        _check_loss_inputs(x, z)
        m = _order_of(x.shape[-1])
        xb = x.reshape(-1, x.shape[-1]).contiguous()
        zb = z.reshape(-1, z.shape[-1]).contiguous()
        p = get_plan(m, xb.shape[0], "r32", x.device)
        num_den = torch.empty(xb.shape[0], m, 2, dtype=torch.float64, device=x.device)
        L = torch.empty((), dtype=torch.float32, device=x.device)
        p.mrdft_spectral_loss_fwd(xb, zb, num_den, L)
        ctx.save_for_backward(xb, zb, num_den)
        ctx.shape = x.shape
        ctx.plan = p
        return L

    @staticmethod
    def backward(ctx, gL):
        xb, zb, num_den = ctx.saved_tensors
        gx = torch.empty_like(xb)
        ctx.plan.mrdft_spectral_loss_bwd(xb, zb, num_den, gL.contiguous().to(torch.float32), gx)
        return gx.reshape(ctx.shape), None


def spectral_loss(x: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
    return SpectralLoss.apply(x, z)


def spectral_loss_terms(x: torch.Tensor, z: torch.Tensor):
    """(num_den (B, m, 2) float64, L) without autograd."""
    _check_loss_inputs(x, z)
    m = _order_of(x.shape[-1])
    xb = x.reshape(-1, x.shape[-1]).contiguous()
    zb = z.reshape(-1, z.shape[-1]).contiguous()
    p = get_plan(m, xb.shape[0], "r32", x.device)
    num_den = torch.empty(xb.shape[0], m, 2, dtype=torch.float64, device=x.device)
    L = torch.empty((), dtype=torch.float32, device=x.device)
    p.mrdft_spectral_loss_fwd(xb, zb, num_den, L)
    return num_den, L
