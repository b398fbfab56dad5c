"""Injected device-allocation failures (MRDFT_FAIL_ALLOC_AT=k): every
allocation site of plan creation, of the first spectral-loss call and of a
2-D plan returns MRDFT_E_ALLOC, sets a message and leaves no device
allocation behind; with the injection off the same calls then work.

Plan creation needs the HIP runtime (device query, uploads), so these run on
the GPU; the failures are injected on the host and no kernel is affected."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import _binding as B
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, log, need_gpu, to_dev, worst_level_err

pytestmark = pytest.mark.gpu


def _live():
    return B.lib().mrdft_live_device_allocations()


@pytest.fixture
def inject():
    old = os.environ.get("MRDFT_FAIL_ALLOC_AT")
    yield
    if old is None:
        os.environ.pop("MRDFT_FAIL_ALLOC_AT", None)
    else:
        os.environ["MRDFT_FAIL_ALLOC_AT"] = old


def _sweep(create, limit=200):
    """Fail allocation k = 1, 2, ... until creation succeeds; returns the number of sites."""
    base = _live()
    for k in range(1, limit):
        os.environ["MRDFT_FAIL_ALLOC_AT"] = str(k)
        try:
            obj = create()
        except B.MrdftError as e:
            assert e.status == B.MRDFT_E_ALLOC, (k, e)
            assert "alloc" in str(e).lower(), (k, str(e))
            assert _live() == base, "allocation %d: %d device allocations leaked" % (k, _live() - base)
            continue
        os.environ.pop("MRDFT_FAIL_ALLOC_AT")
        return k - 1, obj
    raise AssertionError("creation kept failing")


@pytest.mark.parametrize("tune", [False, True])
def test_plan_creation_failures_leak_nothing(inject, tune):
    need_gpu()
    orders = np.array([17, 12, 9, 16, 18, 5], dtype=np.int64)
    off = workloads.offsets_from_orders(orders)
    base = _live()
    sites, plan = _sweep(lambda: api.Plan(offsets=off, dtype="c64", tune=tune))
    log("complex ragged plan (tune=%s): %d allocation sites" % (tune, sites))
    assert sites >= 10
    x = workloads.gaussian_complex(np.random.default_rng(3), int(off[-1]))
    Y = plan.forward(to_dev(x)).cpu().numpy()
    oo = plan.output_offsets()
    for j in (0, 4):
        mj = int(orders[j])
        ref = oracle.forward(x[off[j]:off[j + 1]].astype(np.complex128))
        assert worst_level_err(Y[oo[j]:oo[j + 1]].reshape(mj, -1), ref) <= FWD_TOL
    plan.close()
    assert _live() == base


def test_real_and_half_plans(inject):
    need_gpu()
    base = _live()
    for kw in (dict(m=17, batch=3, dtype="r32"), dict(m=14, batch=2, dtype="r32", half=True)):
        sites, plan = _sweep(lambda: api.Plan(**kw))
        log("plan %s: %d allocation sites" % (kw, sites))
        assert sites >= 5
        plan.close()
    assert _live() == base


@pytest.mark.parametrize("m", [10, 13, 17])
def test_loss_workspace_failures(inject, m):
    """The first loss call allocates the workspace: each of its allocations
    can fail without leaking, and a later call works."""
    need_gpu()
    b = 2
    rng = np.random.default_rng(40 + m)
    x = workloads.gaussian_real(rng, (b, 1 << m))
    z = workloads.gaussian_real(rng, (b, 1 << m))
    xd, zd = to_dev(x), to_dev(z)
    plan = api.Plan(m=m, batch=b, dtype="r32")
    base = _live()
    nd = torch.empty(b, m, 2, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    failed = 0
    for k in range(1, 50):
        os.environ["MRDFT_FAIL_ALLOC_AT"] = str(k)
        try:
            plan.mrdft_spectral_loss_fwd(xd, zd, nd, L)
        except B.MrdftError as e:
            assert e.status == B.MRDFT_E_ALLOC
            assert _live() == base
            failed += 1
            continue
        break
    os.environ.pop("MRDFT_FAIL_ALLOC_AT")
    assert failed >= 2
    torch.cuda.synchronize()
    for s in range(b):
        ndr, _ = oracle.spectral_loss(x[s], z[s])
        assert np.max(np.abs(nd[s].cpu().numpy() / ndr - 1)) <= FWD_TOL
    plan.close()


def test_plan2d_failures(inject):
    need_gpu()
    base = _live()
    sites, p2 = _sweep(lambda: api.Plan2D(6, 5, batch=2, dtype="r32"))
    log("2-D plan: %d allocation sites" % sites)
    assert sites >= 10
    p2.close()
    assert _live() == base
