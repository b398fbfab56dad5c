"""Packed half-spectrum output of real plans against the FP64 oracle (GPU).

Each window of L bins is stored as L/2 values (value 0 = (Y[0], Y[L/2])),
through every kernel that writes a real plan's levels: the one-launch real
forward (4096-sample tiles and the pieces of levels 13..16), the tile kernel
of signals below 4096 samples, and the global passes of the levels above 16.
The adjoint takes the gradient in the same packed layout.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, GRAD_TOL, log, need_gpu, rel_l2, to_dev, worst_level_err

pytestmark = pytest.mark.gpu


def _ragged_real(orders, seed):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum([1 << o for o in orders])]).astype(np.int64)
    return workloads.gaussian_real(rng, (int(offs[-1]),)), offs


@pytest.mark.parametrize("orders,lo,hi", [
    ([2, 3, 4, 5, 9, 11], 1, 28),           # tile kernel only: register and LDS levels
    ([16, 12, 13, 14, 15, 4], 1, 28),       # one-launch real forward, every piece level
    ([17, 12], 1, 28),                      # a pass level above 16
    ([16, 13, 17, 6], 3, 14),               # level range: tiles and pieces only
    ([17, 14], 13, 17),                     # level range: pieces and the pass level
    ([18, 13], 1, 28),                      # two pass levels: one side stream per adjoint chain
    ([18, 17, 12], 1, 28),                  # more pass chains than side streams: one stream
    ([18, 18, 18], 1, 28),                  # adjoint pass chains over window pairs: 3 windows at 18, 6 at 17
])
def test_half_forward_and_adjoint_ragged(orders, lo, hi):
    need_gpu()
    log("half %s [%d, %d]" % (orders, lo, hi))
    x, offs = _ragged_real(orders, 300 + sum(orders) + lo)
    plan = api.Plan(offsets=offs, dtype="r32", levels=(lo, hi), half=True)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(to_dev(x), Y)
    oo = plan.output_offsets()
    Yh = Y.cpu().numpy()
    rng = np.random.default_rng(7 * lo + hi)
    gys = []
    for j, m in enumerate(orders):
        ref = oracle.forward_half(x[offs[j]:offs[j + 1]].astype(np.float64))[lo - 1:min(hi, m)]
        got = Yh[oo[j]:oo[j + 1]].reshape(ref.shape)
        if ref.size:
            assert worst_level_err(got, ref) <= FWD_TOL, (j, m)
        else:
            assert got.size == 0
        gys.append(workloads.gaussian_complex(rng, ref.shape))
    gy = np.concatenate([g.reshape(-1) for g in gys]).astype(np.complex64)
    gx = torch.empty(plan.n_in, dtype=torch.float32, device="cuda")
    plan.mrdft_adjoint(to_dev(gy), gx)
    gxh = gx.cpu().numpy()
    for j, m in enumerate(orders):
        full = np.zeros((m, (1 << m) // 2), dtype=np.complex128)
        if gys[j].size:
            full[lo - 1:lo - 1 + gys[j].shape[0]] = gys[j]
        ref = oracle.adjoint_half(full)
        assert rel_l2(gxh[offs[j]:offs[j + 1]], ref) <= GRAD_TOL, (j, m)


def test_half_uniform_batch_shape_and_values():
    """64 sinusoid mixtures of 2^16 samples, the shape of the real batch
    workload, with half-spectrum output: shape (B, m, N/2), every level
    within the bar on sampled signals, and the same bytes as the full
    output's lower halves."""
    need_gpu()
    rng = np.random.default_rng(1509)
    x = workloads.sinusoid_mix(rng, 64, 1 << 16)
    plan = api.Plan(m=16, batch=64, dtype="r32", half=True)
    xd = to_dev(x)
    Y = plan.forward(xd)
    assert Y.shape == (64, 16, 1 << 15)
    full = api.Plan(m=16, batch=64, dtype="r32").forward(xd)
    for b in (0, 37, 63):
        ref = oracle.forward_half(x[b].astype(np.float64))
        assert worst_level_err(Y[b].cpu().numpy(), ref) <= FWD_TOL, b
    # the packed values are the full output's lower-half bins (same arithmetic)
    for i in (1, 5, 12, 13, 16):
        L = 1 << i
        h = Y[:, i - 1].reshape(64, -1, L // 2).cpu().numpy()
        f = full[:, i - 1].reshape(64, -1, L).cpu().numpy()
        if L > 2:
            assert rel_l2(h[:, :, 1:], f[:, :, 1:L // 2]) <= 1e-7, i
        assert rel_l2(h[:, :, 0].real, f[:, :, 0].real) <= 1e-7, i
        assert rel_l2(h[:, :, 0].imag, f[:, :, L // 2].real) <= 1e-7, i


def test_half_tuned_graph_plan():
    need_gpu()
    rng = np.random.default_rng(1510)
    x = workloads.gaussian_real(rng, (8, 1 << 15))
    plan = api.Plan(m=15, batch=8, dtype="r32", half=True, tune=True, graph=True)
    xd = to_dev(x)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    outs = []
    for _ in range(3):
        Y.zero_()
        plan.mrdft_forward(xd, Y)
        torch.cuda.synchronize()
        outs.append(Y.clone())
    assert all(torch.equal(outs[0], o) for o in outs[1:])
    ref = oracle.forward_half(x[5].astype(np.float64))
    assert worst_level_err(outs[0].view(8, 15, -1)[5].cpu().numpy(), ref) <= FWD_TOL


def test_half_plan_rejects_loss():
    need_gpu()
    plan = api.Plan(m=10, batch=2, dtype="r32", half=True)
    x = torch.randn(2, 1 << 10, device="cuda")
    nd = torch.empty(2, 10, 2, dtype=torch.float64, device="cuda")
    L = torch.empty(1, device="cuda")
    with pytest.raises(RuntimeError, match="full-spectrum"):
        plan.mrdft_spectral_loss_fwd(x, x, nd, L)
