"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _lib():
    from paper_1507_02525_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_1507_02525_amd.build import build
        build()
    return _binding


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(mrdft_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_expected_calls():
    names = declared_functions()
    for n in ("mrdft_plan_create", "mrdft_forward", "mrdft_adjoint", "mrdft_spectral_loss_fwd",
              "mrdft_spectral_loss_bwd", "mrdft_plan_destroy", "mrdft_last_error",
              "mrdft_plan_output_offsets"):
        assert n in names


def test_library_exports_every_declared_symbol():
    b = _lib()
    lib = b.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(b.SIGNATURES)


def _create(b, m, batch, offsets=None, dtype=0, flags=0):
    h = ctypes.c_void_p()
    offp = None
    if offsets is not None:
        arr = np.ascontiguousarray(offsets, dtype=np.int64)
        offp = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    st = b.lib().mrdft_plan_create(ctypes.byref(h), m, batch, offp, dtype, flags, None)
    return st, h


@pytest.mark.parametrize("m,batch,dtype,flags", [(0, 1, 0, 0), (29, 1, 0, 0), (-3, 1, 0, 0), (10, 0, 0, 0),
                                                 (10, -5, 0, 0), (10, 1, 7, 0), (10, 1, 0, 0x80)])
def test_invalid_uniform_arguments(m, batch, dtype, flags):
    b = _lib()
    st, h = _create(b, m, batch, dtype=dtype, flags=flags)
    assert st == b.MRDFT_E_INVALID_ARG
    assert h.value is None
    assert b.last_error() != ""


@pytest.mark.parametrize("offsets", [[1, 5], [0, 3], [0, 4, 4], [0, 8, 4], [0, 2 ** 29]])
def test_invalid_ragged_offsets(offsets):
    b = _lib()
    st, h = _create(b, 0, len(offsets) - 1, offsets=offsets)
    assert st == b.MRDFT_E_INVALID_ARG
    assert h.value is None


def test_ragged_requires_m_zero():
    b = _lib()
    st, _ = _create(b, 5, 1, offsets=[0, 32])
    assert st == b.MRDFT_E_INVALID_ARG


def test_null_and_unknown_handles():
    b = _lib()
    lib = b.lib()
    assert lib.mrdft_plan_create(None, 10, 1, None, 0, 0, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_forward(None, None, None, None) == b.MRDFT_E_INVALID_ARG
    bogus = ctypes.c_void_p(0x1234)
    assert lib.mrdft_forward(bogus, None, None, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_adjoint(bogus, None, None, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan_destroy(bogus) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan_destroy(None) == b.MRDFT_OK
    n = (ctypes.c_int64 * 2)()
    assert lib.mrdft_plan_output_offsets(bogus, n) == b.MRDFT_E_INVALID_ARG
    t, g, o = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.mrdft_plan_schedule(bogus, ctypes.byref(t), ctypes.byref(g), ctypes.byref(o)) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan_schedule(None, None, None, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan_set_schedule(bogus, 11, 1, 0, None) == b.MRDFT_E_INVALID_ARG


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1507_02525_amd import _binding
    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _binding.lib()


@pytest.mark.parametrize("lo,hi", [(0, 5), (6, 5), (1, 29), (11, 12)])
def test_invalid_level_ranges(lo, hi):
    b = _lib()
    h = ctypes.c_void_p()
    st = b.lib().mrdft_plan_create_levels(ctypes.byref(h), 10, 1, None, 0, 0, lo, hi, None)
    assert st == b.MRDFT_E_INVALID_ARG
    assert h.value is None


@pytest.mark.parametrize("m,dtype,offsets", [(10, 0, None),            # complex input
                                             (1, 1, None),             # N = 2 < 4
                                             (0, 1, [0, 8, 10, 26])])  # one ragged signal of 2 samples
def test_invalid_half_spectrum_plans(m, dtype, offsets):
    b = _lib()
    st, h = _create(b, m, 1 if offsets is None else len(offsets) - 1, offsets=offsets, dtype=dtype,
                    flags=b.MRDFT_FLAG_HALF)
    assert st == b.MRDFT_E_INVALID_ARG
    assert h.value is None
    assert "half" in b.last_error()


@pytest.mark.parametrize("m1,m2,batch,dtype", [(0, 4, 1, 0), (4, 0, 1, 1), (29, 2, 1, 0), (24, 20, 1, 0),
                                               (4, 4, 0, 0), (4, 4, 1, 9)])
def test_invalid_2d_plans(m1, m2, batch, dtype):
    b = _lib()
    h = ctypes.c_void_p()
    assert b.lib().mrdft_plan2d_create(ctypes.byref(h), m1, m2, batch, dtype, None) == b.MRDFT_E_INVALID_ARG
    assert h.value is None
    assert b.last_error() != ""


def test_2d_bogus_handles():
    b = _lib()
    lib = b.lib()
    bogus = ctypes.c_void_p(0x1234)
    n = ctypes.c_int64()
    assert lib.mrdft_plan2d_sizes(bogus, ctypes.byref(n), ctypes.byref(n)) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_forward2d(bogus, None, None, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_adjoint2d(bogus, None, None, None) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan2d_destroy(bogus) == b.MRDFT_E_INVALID_ARG
    assert lib.mrdft_plan2d_destroy(None) == b.MRDFT_OK


def test_spectral_loss_rejects_bad_inputs_before_any_call():
    """Shapes, dtypes and devices are checked in Python before the library is
    reached, so a short z can never be read past its end."""
    import torch
    from paper_1507_02525_amd import api
    x = torch.zeros(2, 64)
    with pytest.raises(ValueError):
        api.spectral_loss(x, torch.zeros(2, 32))                 # z shorter than x
    with pytest.raises(ValueError):
        api.spectral_loss(x, torch.zeros(3, 64))                 # batch mismatch
    with pytest.raises(ValueError):
        api.spectral_loss(x, torch.zeros(2, 64))                 # CPU tensors: no CPU path
    with pytest.raises(TypeError):
        api.spectral_loss(x.double(), torch.zeros(2, 64, dtype=torch.float64))
    with pytest.raises(ValueError):
        api.spectral_loss_terms(x, torch.zeros(2, 32))
