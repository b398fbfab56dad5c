"""The paper's rationalised MrDFT, eq. (4), applied factor by factor (FP64 numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

    Y = Gamma * (F^(m) D^(m) A^(m) P^(m)) ... (F^(1) D^(1) A^(1) P^(1)) * X     (eq. 4)

The state is kept as a list of N-long blocks, exactly the blocks the factors
of Section 3 act on:

* P^(1) = 1_{m x 1} (x) I_N copies X into m blocks.
* A^(1) = (I (x) H_2) (+) I applies 2-point Hadamard butterflies to block 1.
* D^(1) multiplies the lower element of each pair by w_2^0 (= 1), F^(1) = I.
* For i >= 2, P^(i) duplicates block i-1, so the state has m+1 blocks;
  A^(i) = I (+) [U^(i) | V^(i)] (+) I folds the duplicate of block i-1 and the
  untouched copy of X (block i) into one block:
    - U^(i), eq. (2): top half of each 2^i window = sum of the two adjacent
      2^(i-1)-long windows of block i-1;
    - V^(i), eq. (3): bottom half = x[n] - x[n + 2^(i-1)] within the window.
* D^(i): bottom half multiplied by diag(w_{2^i}^0 .. w_{2^i}^{2^(i-1)-1}).
* F^(i): bottom half transformed by R_{2^(i-1)} = prod_{j=i-1..1} W^(j) S^(j)
  (S^(1) acts first): S^(j) = I_{2^(j-1)} (x) (H_2 (x) I_{2^(i-j-1)}) is a layer
  of butterflies at distance 2^(i-j-1); W^(j) multiplies the lower half of every
  2^(i-j) block by w_{2^(i-j)}^q, q < 2^(i-j-1).
* Gamma = (+)_i (I (x) T_{2^i}) with (T v)[k] = v[<k>], <k> the i-bit reversal
  (the reading pinned by the printed T_4 and T_8 of Section 4).

Readings taken where the text is garbled: the level block of eq. (1) is
I_{2^(m-i)} (x) E_{2^i}; the superscripts of R^(i) are stage indices j; the
"binary inversion" of the Gamma definition is bit reversal over i bits.

Operation counting (Section 5): every diagonal twiddle entry applied counts as
one complex multiplication (eq. 6); entries equal to w^0 = 1 or w^{n/4} = -j
are "trivial" and excluded from the eq. (7) count; each output of U, V or of
an H_2 butterfly counts one complex addition.
"""
from __future__ import annotations

import numpy as np


def bitrev(v: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (v & 1)
        v >>= 1
    return r


def twiddle(n: int, k) -> np.ndarray:
    """w_n^k = exp(-j 2 pi k / n) in FP64."""
    return np.exp(-2j * np.pi * np.asarray(k, dtype=np.float64) / n)


class Counts:
    def __init__(self, m: int):
        self.mul = [0] * (m + 1)        # all diagonal twiddle entries, per level
        self.mul_nontrivial = [0] * (m + 1)
        self.add = [0] * (m + 1)

    def twiddles(self, level: int, n: int, ks: np.ndarray):
        self.mul[level] += len(ks)
        trivial = (ks == 0) | (4 * ks == n)
        self.mul_nontrivial[level] += int(np.count_nonzero(~trivial))


def _apply_R(v: np.ndarray, i: int, level: int, counts: Counts | None) -> np.ndarray:
    """R_{2^(i-1)} applied to each 2^(i-1)-long row of v (rows = windows)."""
    size = 1 << (i - 1)
    out = v.copy()
    for j in range(1, i):                     # S^(1) first, then W^(1), S^(2), ...
        blk = 1 << (i - j)                    # block length of stage j
        half = blk >> 1
        r = out.reshape(out.shape[0], size // blk, 2, half)
        top = r[:, :, 0, :] + r[:, :, 1, :]   # H_2 (x) I_half
        bot = r[:, :, 0, :] - r[:, :, 1, :]
        q = np.arange(half)
        bot = bot * twiddle(blk, q)[None, None, :]
        if counts is not None:
            counts.add[level] += 2 * half * (size // blk) * out.shape[0]
            counts.twiddles(level, blk, np.tile(q, (size // blk) * out.shape[0]))
        out = np.stack([top, bot], axis=2).reshape(out.shape)
    return out


def mrdft_eq4(x, counts: Counts | None = None) -> np.ndarray:
    """Eq. (4) for one signal x (N = 2^m,) -> (m, N) complex128, natural bin order."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    m = n.bit_length() - 1
    assert n == 1 << m and m >= 1
    # P^(1): m copies of X.
    blocks = [x.copy() for _ in range(m)]
    # A^(1): Hadamard on pairs of block 1; D^(1) = I (+) w_2^0; F^(1) = I.
    pr = blocks[0].reshape(-1, 2)
    b1 = np.empty_like(pr)
    b1[:, 0] = pr[:, 0] + pr[:, 1]
    b1[:, 1] = (pr[:, 0] - pr[:, 1]) * twiddle(2, 0)
    blocks[0] = b1.reshape(-1)
    if counts is not None:
        counts.add[1] += n
        counts.twiddles(1, 2, np.zeros(n // 2, dtype=np.int64))
    for i in range(2, m + 1):
        ln = 1 << i
        h = ln >> 1
        # P^(i): the state becomes [B_1 .. B_{i-1}, B_{i-1}, B_i .. B_m].
        dup = blocks[i - 2].copy()
        xi = blocks[i - 1]                    # still the copy of X made by P^(1)
        # A^(i): [U | V] on (duplicate, X).
        dw = dup.reshape(-1, 2, h)            # two adjacent level-(i-1) windows
        xw = xi.reshape(-1, 2, h)
        top = dw[:, 0, :] + dw[:, 1, :]       # U^(i), eq. (2)
        bot = xw[:, 0, :] - xw[:, 1, :]       # V^(i), eq. (3)
        # D^(i): twiddles w_{2^i}^q on the bottom half.
        q = np.arange(h)
        bot = bot * twiddle(ln, q)[None, :]
        # F^(i): R on the bottom half.
        bot = _apply_R(bot, i, i, counts)
        if counts is not None:
            counts.add[i] += n                # N/2 sums (U) + N/2 differences (V)
            counts.twiddles(i, ln, np.tile(q, n // ln))
        blocks[i - 1] = np.concatenate([top, bot], axis=1).reshape(-1)
    # Gamma: per-window bit reversal of the bin index.
    y = np.empty((m, n), dtype=np.complex128)
    for i in range(1, m + 1):
        ln = 1 << i
        perm = np.array([bitrev(k, i) for k in range(ln)])
        y[i - 1] = blocks[i - 1].reshape(-1, ln)[:, perm].reshape(-1)
    return y


def counts_eq4(m: int) -> Counts:
    c = Counts(m)
    mrdft_eq4(np.zeros(1 << m, dtype=np.complex128), counts=c)
    return c
