"""GPU forward MrDFT vs the FP64 oracle (element by element), all workloads.

Full-size cases that the oracle cannot finish in seconds are checked on
sampled outputs (whole windows of a level, or single bins by direct sums) and
on properties that hold at any size (per-level Parseval).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, GRAD_TOL, log, need_gpu, rel_l2, to_dev, worst_level_err

pytestmark = pytest.mark.gpu


def _api():
    import paper_1507_02525_amd.api as api
    return api


def _check_batch(x_np: np.ndarray, Y: np.ndarray, method=oracle.AUTO, tol=FWD_TOL):
    worst = 0.0
    for b in range(x_np.shape[0]):
        ref = oracle.forward(x_np[b].astype(np.complex128), method)
        worst = max(worst, worst_level_err(Y[b], ref))
    assert worst <= tol, "worst per-level relative L2 %.3e > %.1e" % (worst, tol)
    return worst


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 13, 14, 16])
@pytest.mark.parametrize("dtype", ["c64", "r32"])
def test_forward_small_orders(m, dtype):
    need_gpu()
    log("forward m=%d dtype=%s" % (m, dtype))
    rng = np.random.default_rng(1000 + m)
    b = 3 if m <= 14 else 2
    if dtype == "c64":
        x = workloads.gaussian_complex(rng, (b, 1 << m))
    else:
        x = workloads.gaussian_real(rng, (b, 1 << m))
    Y = _api().forward(to_dev(x)).cpu().numpy()
    assert Y.shape == (b, m, 1 << m)
    w = _check_batch(x, Y)
    log("  worst rel L2 %.3e" % w)


def test_workload1_full():
    need_gpu()
    d = workloads.make(1)
    log("workload 1: c64 m=10")
    Y = _api().forward(to_dev(d["x"])).cpu().numpy()
    w = _check_batch(d["x"], Y, method=oracle.DIRECT)
    log("  worst rel L2 %.3e" % w)


def test_workload2_reduced_batch_all_outputs():
    need_gpu()
    d = workloads.make(2, batch=4)
    log("workload 2 (4 signals): r32 m=16")
    Y = _api().forward(to_dev(d["x"])).cpu().numpy()
    w = _check_batch(d["x"], Y)
    log("  worst rel L2 %.3e" % w)


def test_workload2_full_size_sampled():
    """64 x 2^16 real signals, the benchmark configuration; every level of a
    sample of signals compared with the oracle, all signals by Parseval."""
    need_gpu()
    d = workloads.make(2)
    x = d["x"]
    log("workload 2 full: 64 x r32 m=16")
    Yt = _api().forward(to_dev(x))
    torch.cuda.synchronize()
    for b in (0, 17, 63):
        ref = oracle.forward(x[b].astype(np.complex128))
        w = worst_level_err(Yt[b].cpu().numpy(), ref)
        assert w <= FWD_TOL, (b, w)
    e_x = torch.from_numpy(x.astype(np.float64)).pow(2).sum(1).cuda()
    e_y = Yt.to(torch.complex128).abs().pow(2).sum(2)                 # (B, m)
    lv = torch.pow(2.0, torch.arange(1, 17, device=e_y.device, dtype=torch.float64))
    rel = (e_y / (lv[None, :] * e_x[:, None]) - 1).abs().max().item()
    assert rel < 1e-5, rel


def test_workload3_full_size_sampled():
    """One 2^24 complex signal: top level compared in full with the oracle's
    FFT, window samples of the other levels, direct-sum bins, Parseval."""
    need_gpu()
    d = workloads.make(3)
    x = d["x"][0]
    m = 24
    log("workload 3 full: c64 m=24")
    Yt = _api().forward(to_dev(d["x"]))[0]
    torch.cuda.synchronize()
    # the top level in full
    top = Yt[m - 1].cpu().numpy()
    ref_top = oracle.forward_level(x.astype(np.complex128), m, oracle.FFT)
    assert rel_l2(top, ref_top) <= FWD_TOL
    # a few windows of every level
    x128 = x.astype(np.complex128)
    for i in range(1, m):
        L = 1 << i
        for w in (0, (1 << (m - i)) // 3, (1 << (m - i)) - 1):
            seg = x128[w * L:(w + 1) * L]
            ref = oracle.forward_level(seg, i, oracle.FFT) if i > 1 else np.array([seg[0] + seg[1], seg[0] - seg[1]])
            got = Yt[i - 1, w * L:(w + 1) * L].cpu().numpy()
            assert rel_l2(got, ref) <= FWD_TOL, (i, w, rel_l2(got, ref))
    # direct-sum bins of the two largest levels
    for i in (m - 1, m):
        for (w, k) in ((0, 1), (0, (1 << i) - 1)):
            v = oracle.forward_bin(x128, i, w, k)
            g = complex(Yt[i - 1, w * (1 << i) + k].item())
            scale = np.sqrt(1 << i) * np.sqrt(np.mean(np.abs(x128) ** 2))
            assert abs(g - v) <= 1e-5 * scale
    ex = float(np.sum(np.abs(x128) ** 2))
    ey = Yt.to(torch.complex128).abs().pow(2).sum(1).cpu().numpy()
    for i in range(1, m + 1):
        assert abs(ey[i - 1] / ((1 << i) * ex) - 1) < 1e-5


def test_workload4_ragged_sampled():
    """1000 ragged signals (m in [8, 18]) in one plan; a sample of signals,
    including every order present, compared in full."""
    need_gpu()
    api = _api()
    d = workloads.make(4)
    off = d["offsets"]
    orders = d["orders"]
    log("workload 4 ragged: %d signals, %d samples" % (len(orders), off[-1]))
    p = api.Plan(offsets=off, dtype="c64")
    Y = p.forward(to_dev(d["x"])).cpu().numpy()
    oo = p.output_offsets()
    pick = set([0, len(orders) - 1])
    for o in np.unique(orders):
        pick.add(int(np.nonzero(orders == o)[0][0]))
    for j in sorted(pick):
        mj = int(orders[j])
        n = 1 << mj
        xs = d["x"][off[j]:off[j + 1]].astype(np.complex128)
        ref = oracle.forward(xs)
        got = Y[oo[j]:oo[j + 1]].reshape(mj, n)
        assert worst_level_err(got, ref) <= FWD_TOL, (j, mj)


def test_ragged_mixed_small_orders():
    """Ragged batch mixing every order 1..14 (odd offsets for real data, tiles
    smaller than 16 samples, upper levels)."""
    need_gpu()
    api = _api()
    rng = np.random.default_rng(77)
    orders = np.array([1, 3, 2, 14, 1, 5, 13, 4, 6, 12, 7, 8, 9, 10, 11, 2, 1], dtype=np.int64)
    off = workloads.offsets_from_orders(orders)
    for dtype in ("c64", "r32"):
        x = workloads.gaussian_complex(rng, int(off[-1])) if dtype == "c64" else \
            workloads.gaussian_real(rng, int(off[-1]))
        p = api.Plan(offsets=off, dtype=dtype)
        Y = p.forward(to_dev(x)).cpu().numpy()
        oo = p.output_offsets()
        for j, mj in enumerate(orders):
            ref = oracle.forward(x[off[j]:off[j + 1]].astype(np.complex128))
            got = Y[oo[j]:oo[j + 1]].reshape(int(mj), -1)
            assert worst_level_err(got, ref) <= FWD_TOL, (dtype, j, mj)


def test_zero_and_impulse_inputs():
    need_gpu()
    api = _api()
    m = 13
    x = torch.zeros(2, 1 << m, dtype=torch.complex64, device="cuda")
    Y = api.forward(x)
    assert torch.count_nonzero(Y).item() == 0
    x[1, 5] = 1.0
    Y = api.forward(x).cpu().numpy()
    ref = oracle.forward(x[1].cpu().numpy().astype(np.complex128))
    assert worst_level_err(Y[1], ref) <= FWD_TOL
    assert np.count_nonzero(Y[0]) == 0


def test_repeat_runs_bitwise_identical():
    need_gpu()
    api = _api()
    d = workloads.make(2, batch=8)
    xt = to_dev(d["x"])
    a = api.forward(xt)
    b = api.forward(xt)
    assert torch.equal(a, b)


def test_maximum_order_sampled():
    """One real signal of 2^28 samples (the largest order; 60 GB of output):
    direct-sum bins of the top level, windows of lower levels against the
    oracle's FFT route, per-level Parseval, and A^H A x = (2^(m+1) - 2) x
    through the adjoint."""
    need_gpu()
    m = 28
    log("maximum order: r32 m=28")
    rng = np.random.default_rng(1528)
    x = rng.standard_normal(1 << m, dtype=np.float32)
    xd = to_dev(x)
    plan = api.Plan(m=m, batch=1, dtype="r32")
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(xd, Y)
    torch.cuda.synchronize()
    Yl = Y.view(m, 1 << m)
    rms = float(np.sqrt(np.mean(x.astype(np.float64) ** 2)))
    for i, w, k in ((m, 0, 1), (m, 0, (1 << m) - 3), (m - 1, 1, 12345), (20, 77, 999)):
        L = 1 << i
        seg = x[w * L:(w + 1) * L].astype(np.float64)
        v = oracle.forward_bin(seg, i, 0, k)
        g = complex(Yl[i - 1, w * L + k].item())
        assert abs(g - v) <= 1e-5 * np.sqrt(L) * rms, (i, w, k, g, v)
    for i, w in ((1, 5), (12, 3), (13, 1000), (16, 4095), (17, 7), (20, 100)):
        L = 1 << i
        seg = x[w * L:(w + 1) * L].astype(np.complex128)
        ref = oracle.forward_level(seg, i, oracle.FFT) if i > 1 else np.array([seg[0] + seg[1], seg[0] - seg[1]])
        got = Yl[i - 1, w * L:(w + 1) * L].cpu().numpy()
        assert rel_l2(got, ref) <= FWD_TOL, (i, w, rel_l2(got, ref))
    ex = float(torch.sum(xd.double() ** 2).item())
    for i in range(1, m + 1):
        ey = float(torch.sum(Yl[i - 1].abs().double() ** 2).item())
        assert abs(ey / ((1 << i) * ex) - 1) < 1e-5, i
    gx = torch.empty_like(xd)
    plan.mrdft_adjoint(Y, gx)
    del Y, Yl
    scale = float((1 << (m + 1)) - 2)
    err = torch.linalg.vector_norm((gx.double() - scale * xd.double())).item() / (scale * np.sqrt(ex))
    assert err <= GRAD_TOL, err
