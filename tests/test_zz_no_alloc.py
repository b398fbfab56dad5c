"""mrdft_spectral_loss_fwd_noalloc (no device allocation, library-held
workspace) against mrdft_spectral_loss_fwd on the same inputs, through the C
ABI: two calls in a row, the second on a smaller input; the FP64 oracle
checks both; the library's device allocations do not change; sizes beyond the
workspace and unsupported plans are refused with a message."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import _binding as B
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, log, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(batch, m, seed):
    rng = np.random.default_rng(seed)
    return workloads.gaussian_real(rng, (batch, 1 << m)), workloads.gaussian_real(rng, (batch, 1 << m))


def test_noalloc_matches_allocating_entry_point():
    need_gpu()
    lib = B.lib()
    for batch, m, seed in ((8, 16, 71), (3, 13, 72)):              # the second call: a smaller input
        log("noalloc loss forward batch=%d m=%d" % (batch, m))
        x, z = _case(batch, m, seed)
        xd, zd = to_dev(x), to_dev(z)
        plan = api.Plan(m=m, batch=batch, dtype="r32")
        nd_a = torch.full((batch, m, 2), -1.0, dtype=torch.float64, device="cuda")
        L_a = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
        live = lib.mrdft_live_device_allocations()
        B.check(lib.mrdft_spectral_loss_fwd_noalloc(plan.handle, _p(xd), _p(zd), _p(nd_a), _p(L_a), _stream()))
        torch.cuda.synchronize()
        assert lib.mrdft_live_device_allocations() == live, "the no-allocation entry point allocated"
        nd_b = torch.empty_like(nd_a)
        L_b = torch.empty_like(L_a)
        B.check(lib.mrdft_spectral_loss_fwd(plan.handle, _p(xd), _p(zd), _p(nd_b), _p(L_b), _stream()))
        torch.cuda.synchronize()
        a, b_ = nd_a.cpu().numpy(), nd_b.cpu().numpy()
        assert np.max(np.abs(a / b_ - 1)) <= FWD_TOL
        assert abs(L_a.item() / L_b.item() - 1) <= FWD_TOL
        Lref = 0.0
        for s in range(batch):
            ndr, lr = oracle.spectral_loss(x[s], z[s])
            assert np.max(np.abs(a[s] / ndr - 1)) <= FWD_TOL, s
            Lref += lr
        assert abs(L_a.item() / Lref - 1) <= FWD_TOL
        plan.close()


def test_noalloc_refuses_what_it_cannot_hold():
    need_gpu()
    lib = B.lib()
    nd = torch.empty(1, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    x = torch.empty(1 << 17, dtype=torch.float32, device="cuda")
    for kw in (dict(m=17, batch=1, dtype="r32"),        # order above the one-launch levels
               dict(m=11, batch=1, dtype="r32"),        # below the real tile
               dict(m=12, batch=1, dtype="c64"),        # complex plan
               dict(m=12, batch=2731, dtype="r32")):    # batch * m beyond the workspace
        plan = api.Plan(**kw)
        st = lib.mrdft_spectral_loss_fwd_noalloc(plan.handle, _p(x), _p(x), _p(nd), _p(L), _stream())
        assert st == B.MRDFT_E_UNSUPPORTED, kw
        assert "noalloc" in B.last_error() or "spectral loss" in B.last_error()
        plan.close()
