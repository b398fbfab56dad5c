"""Seeded synthetic inputs for the multiresolution DFT.

This module only draws numbers: it holds none of the transform's arithmetic.
Both the FP64 oracle (through the tests) and the GPU path take their inputs
from here, so the two sides always see identical float32 / complex64 data.

Every draw is made in float64 with ``numpy.random.default_rng(1507 + k)``
(k = workload number below) and then rounded once to float32 / complex64.

Workloads (the signal model follows the problem statement of Section 2:
one signal of N = 2^m samples, transformed at every level i = 1..m):

1. one complex64 signal, m = 10, real and imaginary parts i.i.d. N(0, 1);
2. 64 real float32 signals, m = 16, each a sum of 8 sinusoids
   a*cos(2*pi*f*n + phi) with f ~ U[0, 0.5), a ~ U(0.1, 1), phi ~ U(0, 2*pi),
   plus 0.1 * N(0, 1) noise;
3. one complex64 signal, m = 24, i.i.d. N(0, 1) parts;
4. 1000 complex64 signals of lengths 2^m_j with m_j uniform on {8, ..., 18},
   packed back to back and described by an int64 offsets array;
5. 32 real float32 pairs (x, z), m = 18, both i.i.d. N(0, 1).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1507


def rng_for(k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(k))


def gaussian_complex(rng: np.random.Generator, shape) -> np.ndarray:
    """complex64 with i.i.d. N(0,1) real and imaginary parts (drawn in float64)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex64)


def gaussian_real(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape).astype(np.float32)


def sinusoid_mix(rng: np.random.Generator, batch: int, n: int, tones: int = 8,
                 noise: float = 0.1) -> np.ndarray:
    """float32 signals: sum of `tones` random cosines plus Gaussian noise."""
    t = np.arange(n, dtype=np.float64)
    out = np.empty((batch, n), dtype=np.float32)
    for b in range(batch):
        f = rng.uniform(0.0, 0.5, tones)
        a = rng.uniform(0.1, 1.0, tones)
        phi = rng.uniform(0.0, 2.0 * np.pi, tones)
        s = (a[:, None] * np.cos(2.0 * np.pi * f[:, None] * t[None, :] + phi[:, None])).sum(0)
        s += noise * rng.standard_normal(n)
        out[b] = s.astype(np.float32)
    return out


def ragged_orders(rng: np.random.Generator, count: int, m_lo: int, m_hi: int) -> np.ndarray:
    """int64 array of per-signal orders m_j, uniform on {m_lo, ..., m_hi}."""
    return rng.integers(m_lo, m_hi + 1, size=count).astype(np.int64)


def offsets_from_orders(orders: np.ndarray) -> np.ndarray:
    """Sample offsets [batch+1] (int64, starting at 0) for signals of length 2^m_j."""
    lens = np.left_shift(np.int64(1), orders.astype(np.int64))
    off = np.zeros(len(orders) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


# Workload table.  `scale` shrinks the batch (and, for the ragged case, the
# signal count and maximum order) so parity tests can run the oracle quickly
# on inputs of the same kind.
WORKLOADS = {
    1: dict(name="c64 single signal m=10", m=10, batch=1, dtype="c64"),
    2: dict(name="64 x r32 sinusoid mixes m=16", m=16, batch=64, dtype="r32"),
    3: dict(name="c64 single long signal m=24", m=24, batch=1, dtype="c64"),
    4: dict(name="ragged 1000 x c64, m in [8,18]", m_lo=8, m_hi=18, count=1000, dtype="c64"),
    5: dict(name="spectral loss 32 x r32 pairs m=18", m=18, batch=32, dtype="r32"),
}


def make(k: int, batch: int | None = None, m: int | None = None,
         count: int | None = None, m_hi: int | None = None) -> dict:
    """Draw workload k.  Optional arguments override its size (same recipe)."""
    spec = dict(WORKLOADS[k])
    rng = rng_for(k)
    if k == 4:
        cnt = count if count is not None else spec["count"]
        hi = m_hi if m_hi is not None else spec["m_hi"]
        lo = min(spec["m_lo"], hi)
        orders = ragged_orders(rng, cnt, lo, hi)
        off = offsets_from_orders(orders)
        x = gaussian_complex(rng, int(off[-1]))
        return dict(k=k, dtype="c64", orders=orders, offsets=off, x=x, batch=cnt)
    mm = m if m is not None else spec["m"]
    b = batch if batch is not None else spec["batch"]
    n = 1 << mm
    out = dict(k=k, m=mm, batch=b, dtype=spec["dtype"])
    if k in (1, 3):
        out["x"] = gaussian_complex(rng, (b, n))
    elif k == 2:
        out["x"] = sinusoid_mix(rng, b, n)
    elif k == 5:
        out["x"] = gaussian_real(rng, (b, n))
        out["z"] = gaussian_real(rng, (b, n))
    return out
