"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies ``oracle/mrdft_oracle.c``, plants one plausible mistake (a
sign, an index, a dropped term, a swapped operand), builds the copy with gcc
into a temporary directory and runs the pin battery through it.  At least one
pin has to fail for every mutant, and none may fail for the unmodified source.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import dense_eq1, rand_c, w

SRC = os.path.join(os.path.dirname(oracle.__file__), "mrdft_oracle.c")

MUTANTS = {
    "twiddle_sign": ("t[e].im = -sin(a);", "t[e].im = sin(a);"),
    "exponent_mask": ("tw[(n * k) & mask])", "tw[(n * k) & (mask >> 1)])"),
    "dropped_last_term": ("for (int64_t n = 0; n < len; ++n)\n                acc = c_add(acc, c_mul(x[base + n]",
                          "for (int64_t n = 0; n < len - 1; ++n)\n                acc = c_add(acc, c_mul(x[base + n]"),
    "butterfly_swapped": ("out[k] = c_add(e, o);\n        out[k + h] = c_sub(e, o);",
                          "out[k] = c_sub(e, o);\n        out[k + h] = c_add(e, o);"),
    "fft_twiddle_index": ("c_mul(out[k + h], tw[k * tws])", "c_mul(out[k + h], tw[k])"),
    "adjoint_no_conj": ("c_mul(gy[base + k], c_conj(tw[(n * k) & mask]))",
                        "c_mul(gy[base + k], tw[(n * k) & mask])"),
    "adjoint_fft_no_conj_out": ("gx[base + n] = c_add(gx[base + n], c_conj(b[n]));",
                                "gx[base + n] = c_add(gx[base + n], b[n]);"),
    "bin_window_offset": ("const cplx *xs = (const cplx *)x + w * len;",
                          "const cplx *xs = (const cplx *)x + w * (len / 2);"),
    "loss_ratio_inverted": ("total += num / den;", "total += den / num;"),
    "grad_scale_dropped_2": ("const double s = gL * 2.0 /", "const double s = gL * 1.0 /"),
    "level_stack_offset": ("y + 2 * (size_t)(i - 1) * (size_t)n_all", "y + 2 * (size_t)(m - i) * (size_t)n_all"),
}


def pin_failures():
    """Compact pin battery; returns the names of failing pins."""
    bad = []
    rng = np.random.default_rng(5)
    for m in (3, 5):
        x = rand_c(rng, 1 << m)
        ref = (dense_eq1(m) @ x).reshape(m, -1)
        for method in (oracle.DIRECT, oracle.FFT):
            if np.max(np.abs(oracle.forward(x, method) - ref)) > 1e-10:
                bad.append("dense_eq1_m%d_method%d" % (m, method))
        gy = rand_c(rng, m << m).reshape(m, -1)
        aref = dense_eq1(m).conj().T @ gy.reshape(-1)
        for method in (oracle.DIRECT, oracle.FFT):
            if np.max(np.abs(oracle.adjoint(gy, method) - aref)) > 1e-10:
                bad.append("dense_adjoint_m%d_method%d" % (m, method))
        for p in (0, (1 << m) - 1):
            if abs(oracle.adjoint_point(gy, p) - aref[p]) > 1e-10:
                bad.append("adjoint_point_m%d" % m)
        for i in (1, m):
            L = 1 << i
            wi = (1 << (m - i)) - 1
            if abs(oracle.forward_bin(x, i, wi, L - 1) - ref[i - 1][wi * L + L - 1]) > 1e-10:
                bad.append("bin_m%d_i%d" % (m, i))
    m = 6
    xr = rng.standard_normal(1 << m)
    zr = rng.standard_normal(1 << m)
    nd, L = oracle.spectral_loss(xr, zr)
    ratio = np.sum((xr - zr) ** 2) / np.sum(zr ** 2)
    if abs(L - ratio) > 1e-10 * ratio:
        bad.append("loss_closed_form")
    g = oracle.spectral_loss_grad(xr, zr, nd)
    if np.max(np.abs(g - 2 * (xr - zr) / np.sum(zr ** 2))) > 1e-10:
        bad.append("grad_closed_form")
    # impulse closed form at the top level
    x = np.zeros(1 << m, dtype=np.complex128)
    x[5] = 1
    if np.max(np.abs(oracle.forward(x)[m - 1] - w(1 << m, 5 * np.arange(1 << m)))) > 1e-12:
        bad.append("impulse")
    return bad


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new, 1)
    cpath = tmp_path / ("%s.c" % name)
    cpath.write_text(mutated)
    so = tmp_path / ("lib%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                           "-o", str(so), str(cpath), "-lm"])
    return str(so)


def test_unmodified_source_passes_battery():
    assert pin_failures() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    so = _build_variant(tmp_path, name, old, new)
    with oracle.use_library(so):
        failed = pin_failures()
    assert failed, "planted mistake %s was not caught by any pin" % name
