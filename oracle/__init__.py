"""FP64 CPU oracle for the multiresolution DFT — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and the
two share no code: the only thing both sides use is the seeded input module
``paper_1507_02525_amd.workloads``, which draws numbers and computes nothing.

Contents
  * ``mrdft_oracle.c`` (built into ``libmrdft_oracle.so``): the definition of
    eq. (1) written out as direct per-window sums, a plain recursive radix-2
    FFT per window, the conjugate-transpose (adjoint), single-output direct
    sums for sampling huge transforms, and the spectral loss and its gradient.
  * ``recurrence.py``: the paper's rationalised factorisation, eq. (4),
    applied factor by factor in FP64 numpy, with operation counting (Section 5).

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against things other than itself (dense Kronecker matrices of eq. (1), the
printed permutations T_4 / T_8 of Section 4, numpy.fft as an independent
library FFT, closed forms, Parseval, adjoint identities and the counts of
eqs. (6)-(7)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrdft_oracle.c")
_LIB = os.path.join(_HERE, "libmrdft_oracle.so")
_lib = None

DIRECT, FFT, AUTO = 0, 1, -1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.mro_forward_level.argtypes = [ci, ci, dp, dp, ci]
    lib.mro_forward.argtypes = [ci, dp, dp, ci]
    lib.mro_forward_bin.argtypes = [ci, ci, i64, i64, dp, dp]
    lib.mro_adjoint.argtypes = [ci, dp, dp, ci]
    lib.mro_adjoint_point.argtypes = [ci, i64, dp, dp]
    lib.mro_spectral_loss.argtypes = [ci, dp, dp, dp, dp, ci]
    lib.mro_spectral_loss_grad.argtypes = [ci, dp, dp, dp, ctypes.c_double, dp, ci]
    for f in (lib.mro_forward_level, lib.mro_forward, lib.mro_forward_bin, lib.mro_adjoint,
              lib.mro_adjoint_point, lib.mro_spectral_loss, lib.mro_spectral_loss_grad):
        f.restype = ci
    return lib


class use_library:
    """Context manager: route the wrappers through another build of the C
    source (the mutation tests plant mistakes in a copy and check that the
    pins catch them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(_LIB)
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex128)


def _order(n: int) -> int:
    m = int(n).bit_length() - 1
    if n < 2 or (1 << m) != n:
        raise ValueError("signal length must be 2^m with m >= 1, got %d" % n)
    return m


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError("oracle %s failed (rc=%d)" % (what, rc))


def forward(x, method: int = AUTO) -> np.ndarray:
    """All levels of one signal: x (N,) -> complex128 (m, N)."""
    xc = _c128(x)
    m = _order(xc.size)
    y = np.empty((m, xc.size), dtype=np.complex128)
    _check(_load().mro_forward(m, _dp(xc), _dp(y), method), "forward")
    return y


def forward_level(x, i: int, method: int = AUTO) -> np.ndarray:
    """Level i (1-based) of one signal: x (N,) -> complex128 (N,)."""
    xc = _c128(x)
    m = _order(xc.size)
    y = np.empty(xc.size, dtype=np.complex128)
    _check(_load().mro_forward_level(m, int(i), _dp(xc), _dp(y), method), "forward_level")
    return y


def forward_bin(x, i: int, w: int, k: int) -> complex:
    """Single output Y^(i)[w*2^i + k] by its direct sum."""
    xc = _c128(x)
    m = _order(xc.size)
    out = np.empty(2, dtype=np.float64)
    _check(_load().mro_forward_bin(m, int(i), int(w), int(k), _dp(xc), _dp(out)), "forward_bin")
    return complex(out[0], out[1])


def adjoint(gy, method: int = AUTO) -> np.ndarray:
    """gy (m, N) -> complex128 (N,): sum over levels of per-window conjugate DFTs."""
    g = _c128(gy)
    m, n = g.shape
    if _order(n) != m:
        raise ValueError("gy must have shape (m, 2^m)")
    gx = np.empty(n, dtype=np.complex128)
    _check(_load().mro_adjoint(m, _dp(g), _dp(gx), method), "adjoint")
    return gx


def adjoint_point(gy, p: int) -> complex:
    g = _c128(gy)
    m, n = g.shape
    out = np.empty(2, dtype=np.float64)
    _check(_load().mro_adjoint_point(m, int(p), _dp(g), _dp(out)), "adjoint_point")
    return complex(out[0], out[1])


def spectral_loss(x, z, method: int = AUTO):
    """Real signals x, z (N,) -> (num_den (m, 2) float64, L float)."""
    xr = np.ascontiguousarray(x, dtype=np.float64)
    zr = np.ascontiguousarray(z, dtype=np.float64)
    m = _order(xr.size)
    nd = np.empty((m, 2), dtype=np.float64)
    loss = np.empty(1, dtype=np.float64)
    _check(_load().mro_spectral_loss(m, _dp(xr), _dp(zr), _dp(nd), _dp(loss), method),
           "spectral_loss")
    return nd, float(loss[0])


def spectral_loss_grad(x, z, num_den, gL: float = 1.0, method: int = AUTO) -> np.ndarray:
    xr = np.ascontiguousarray(x, dtype=np.float64)
    zr = np.ascontiguousarray(z, dtype=np.float64)
    nd = np.ascontiguousarray(num_den, dtype=np.float64)
    m = _order(xr.size)
    gx = np.empty(xr.size, dtype=np.float64)
    _check(_load().mro_spectral_loss_grad(m, _dp(xr), _dp(zr), _dp(nd), float(gL), _dp(gx),
                                          method), "spectral_loss_grad")
    return gx


# ---------------------------------------------------------------------------
# Packed half-spectrum layout of a real signal's levels.  The paper does not
# treat real input; this is the plain definition of the optional output: a
# real window's spectrum is Hermitian (Y[L-k] = conj(Y[k])), so window w of a
# level with L-point windows keeps L/2 values: value 0 = (Re Y[0], Re Y[L/2])
# packed as one complex number, value k = Y[k] for 0 < k < L/2.

def pack_half(Y) -> np.ndarray:
    """Full levels (m, N) of a real signal -> packed half spectra (m, N/2)."""
    Y = _c128(Y)
    m, n = Y.shape
    out = np.empty((m, n // 2), dtype=np.complex128)
    for i in range(1, m + 1):
        L = 1 << i
        win = Y[i - 1].reshape(n // L, L)
        h = out[i - 1].reshape(n // L, L // 2)
        h[:, 0] = win[:, 0].real + 1j * win[:, L // 2].real
        h[:, 1:] = win[:, 1:L // 2]
    return out


def unpack_half_zero(gh) -> np.ndarray:
    """Packed (m, N/2) -> full (m, N): value 0 back to bins 0 and L/2 as real
    numbers, value k to bin k, every bin above L/2 zero (the transpose of
    pack_half as a real-linear map)."""
    gh = _c128(gh)
    m, h = gh.shape
    n = 2 * h
    out = np.zeros((m, n), dtype=np.complex128)
    for i in range(1, m + 1):
        L = 1 << i
        src = gh[i - 1].reshape(n // L, L // 2)
        dst = out[i - 1].reshape(n // L, L)
        dst[:, 0] = src[:, 0].real
        dst[:, L // 2] = src[:, 0].imag
        dst[:, 1:L // 2] = src[:, 1:]
    return out


def forward_half(x, method: int = AUTO) -> np.ndarray:
    """Real x (N,) -> packed half spectra of every level, complex128 (m, N/2)."""
    xr = np.asarray(x)
    if np.iscomplexobj(xr):
        raise ValueError("the half-spectrum layout is defined for real signals")
    return pack_half(forward(xr.astype(np.float64), method))


def adjoint_half(gh, method: int = AUTO) -> np.ndarray:
    """Gradient of a real loss of the packed values with respect to real x:
    Re(A^H unpack_half_zero(gh)), float64 (N,)."""
    return adjoint(unpack_half_zero(gh), method).real


# ---------------------------------------------------------------------------
# Two-dimensional separable MrDFT (the paper names two-dimensional signals as
# an application and gives no formula).  Reading: for an image x of
# N1 x N2 = 2^m1 x 2^m2 samples and every pair of levels (i1, i2), the 2-D DFT
# of every non-overlapping 2^i1 x 2^i2 block,
#   Y[i1, i2][b1 L1 + k1, b2 L2 + k2] =
#       sum_{n1 < L1, n2 < L2} x[b1 L1 + n1, b2 L2 + n2] w_L1^{n1 k1} w_L2^{n2 k2},
# i.e. Y[i1, i2] = A1_i1 x A2_i2^T with A_i the level-i block of eq. (1).
# Being separable, it is computed here with the 1-D oracle along the rows and
# then along the columns (the pins check it against the double sum itself).

def forward2d(x, method: int = AUTO) -> np.ndarray:
    """Image x (N1, N2) -> complex128 (m1, m2, N1, N2)."""
    xc = _c128(x)
    if xc.ndim != 2:
        raise ValueError("x must be a 2-D array")
    n1, n2 = xc.shape
    m1, m2 = _order(n1), _order(n2)
    rows = np.stack([forward(xc[r], method) for r in range(n1)])          # (N1, m2, N2)
    out = np.empty((m1, m2, n1, n2), dtype=np.complex128)
    for i2 in range(m2):
        for c in range(n2):
            out[:, i2, :, c] = forward(rows[:, i2, c], method)              # (m1, N1)
    return out


def adjoint2d(gy, method: int = AUTO) -> np.ndarray:
    """gy (m1, m2, N1, N2) -> complex128 (N1, N2): the conjugate transpose of
    forward2d, sum over level pairs of A1_i1^H gy[i1, i2] conj(A2_i2)."""
    g = _c128(gy)
    m1, m2, n1, n2 = g.shape
    if _order(n1) != m1 or _order(n2) != m2:
        raise ValueError("gy must have shape (m1, m2, 2^m1, 2^m2)")
    part = np.empty((m2, n1, n2), dtype=np.complex128)
    for i2 in range(m2):
        for c in range(n2):
            part[i2, :, c] = adjoint(g[:, i2, :, c], method)                # columns first
    return np.stack([adjoint(part[:, r, :], method) for r in range(n1)])
