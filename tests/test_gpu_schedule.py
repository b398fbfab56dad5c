"""Schedules of the forward launch against the FP64 oracle (GPU).

Covers the complex launch (one workgroup per job, or persistent with any
grid, including a single workgroup
that takes every job), each job order, the tile kernel with one launch per
upper level, the tuner's choice, the queue that the persistent launch leaves
cleared for the next call, and graph replay against eager calls.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, log, need_gpu, to_dev, worst_level_err

pytestmark = pytest.mark.gpu

ORDERS = ("tiles_first", "rows_first", "interleaved", "blocks")


def _ragged(orders, seed, dtype="c64"):
    rng = np.random.default_rng(seed)
    n = [1 << o for o in orders]
    offs = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    if dtype == "c64":
        x = workloads.gaussian_complex(rng, (int(offs[-1]),))
    else:
        x = workloads.gaussian_real(rng, (int(offs[-1]),))
    return x, offs


def _check_ragged(Y, x, offs, orders, plan):
    oo = plan.output_offsets()
    Yh = Y.cpu().numpy()
    worst = 0.0
    for j, m in enumerate(orders):
        N = 1 << m
        ref = oracle.forward(x[offs[j]:offs[j + 1]].astype(np.complex128))
        got = Yh[oo[j]:oo[j + 1]].reshape(m, N)
        worst = max(worst, worst_level_err(got, ref))
    return worst


# orders around every boundary: tile sizes 2^11 / 2^12, upper pieces up to 2^16, passes above
C_ORDERS = [11, 12, 9, 13, 14, 16, 17, 15, 5, 12]


@pytest.mark.parametrize("tile_log,grid,order", [(11, 0, "tiles_first"), (11, 0, "interleaved"),
                                                 (11, 1, "tiles_first"), (11, 7, "rows_first"),
                                                 (11, 1024, "interleaved"), (11, 256, "tiles_first"),
                                                 (12, 0, "tiles_first"), (11, 0, "blocks"), (11, 512, "blocks")])
def test_complex_schedules_match_oracle(tile_log, grid, order):
    need_gpu()
    log("complex schedule tile_log=%d grid=%d order=%s" % (tile_log, grid, order))
    x, offs = _ragged(C_ORDERS, 41)
    plan = api.Plan(offsets=offs, dtype="c64")
    plan.set_schedule(tile_log, grid, order)
    assert plan.schedule() == {"tile_log": tile_log, "grid": grid if tile_log == 11 else 0, "order": order,
                               "serial": False, "after": False}
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(to_dev(x), Y)
    err = _check_ragged(Y, x, offs, C_ORDERS, plan)
    log("  worst rel err %.3e" % err)
    assert err <= FWD_TOL


@pytest.mark.parametrize("order", ORDERS)
def test_real_orders_match_oracle(order):
    need_gpu()
    orders = [12, 16, 13, 8, 14, 15]
    log("real order %s" % order)
    x, offs = _ragged(orders, 43, dtype="r32")
    plan = api.Plan(offsets=offs, dtype="r32")
    plan.set_schedule(12, 0, order)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(to_dev(x), Y)
    err = _check_ragged(Y, x, offs, orders, plan)
    log("  worst rel err %.3e" % err)
    assert err <= FWD_TOL


def test_persistent_queue_is_reusable():
    """Each call of the persistent launch must find the job queue cleared by
    the previous one: repeated calls into a zeroed Y give identical results."""
    need_gpu()
    x, offs = _ragged([13, 11, 14, 12], 45)
    plan = api.Plan(offsets=offs, dtype="c64")
    plan.set_schedule(11, 3, "tiles_first")
    xd = to_dev(x)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    first = None
    for it in range(5):
        Y.zero_()
        plan.mrdft_forward(xd, Y)
        cur = Y.cpu()
        if first is None:
            first = cur
            assert _check_ragged(Y, x, offs, [13, 11, 14, 12], plan) <= FWD_TOL
        else:
            assert torch.equal(cur, first), "call %d differs" % it


@pytest.mark.parametrize("dtype", ["c64", "r32"])
def test_graph_replay_matches_eager(dtype):
    need_gpu()
    orders = [14, 12, 16, 10] if dtype == "c64" else [12, 16, 14]
    log("graph replay %s" % dtype)
    xs = [_ragged(orders, 50 + k, dtype=dtype)[0] for k in range(3)]
    offs = _ragged(orders, 50, dtype=dtype)[1]
    eager = api.Plan(offsets=offs, dtype=dtype)
    graphed = api.Plan(offsets=offs, dtype=dtype, graph=True)
    xd = to_dev(xs[0])
    Yg = torch.empty(eager.n_out, dtype=torch.complex64, device="cuda")
    Ye = torch.empty_like(Yg)
    for k in range(3):
        xd.copy_(to_dev(xs[k]))              # same pointers, new contents
        Yg.zero_()
        graphed.mrdft_forward(xd, Yg)        # first call captures, later calls replay
        junk = torch.randn(1 << 20, device="cuda") * 2.0     # eager work between replays
        eager.mrdft_forward(xd, Ye)
        torch.cuda.synchronize()
        assert torch.equal(Yg, Ye), "replay %d differs from the eager call" % k
        del junk
    assert _check_ragged(Yg, xs[2], offs, orders, graphed) <= FWD_TOL


def test_tuned_plan_matches_oracle():
    need_gpu()
    d = workloads.make(4, count=60, m_hi=17)
    x, offs = d["x"], d["offsets"]
    orders = [int(np.log2(offs[j + 1] - offs[j])) for j in range(len(offs) - 1)]
    plan = api.Plan(offsets=offs, dtype="c64", tune=True)
    sch = plan.schedule()
    log("tuned schedule %s" % sch)
    assert sch["tile_log"] in (11, 12) and sch["order"] in ORDERS
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(to_dev(x), Y)
    # sampled: the 6 largest and 6 random signals
    oo = plan.output_offsets()
    Yh = Y.cpu().numpy()
    rng = np.random.default_rng(7)
    pick = list(np.argsort(orders)[-6:]) + list(rng.choice(len(orders), 6, replace=False))
    for j in pick:
        m = orders[j]
        ref = oracle.forward(x[offs[j]:offs[j + 1]].astype(np.complex128))
        err = worst_level_err(Yh[oo[j]:oo[j + 1]].reshape(m, 1 << m), ref)
        assert err <= FWD_TOL, (j, m, err)




@pytest.mark.parametrize("mode", ["beside", "serial", "after"])
def test_stream_modes_match_oracle(mode):
    """The levels above the one-launch kernel on side streams beside it, all
    on the caller's stream, or on side streams after it: the same result
    (bit for bit) and the oracle's, eager and under graph replay."""
    need_gpu()
    orders = [17, 12, 18, 9, 17, 16]
    x, offs = _ragged(orders, 61)
    ref = api.Plan(offsets=offs, dtype="c64")
    Yr = torch.empty(ref.n_out, dtype=torch.complex64, device="cuda")
    xd = to_dev(x)
    ref.mrdft_forward(xd, Yr)
    for graph in (False, True):
        plan = api.Plan(offsets=offs, dtype="c64", graph=graph)
        plan.set_schedule(11, 0, "blocks", mode == "serial", mode == "after")
        sch = plan.schedule()
        assert sch["serial"] == (mode == "serial") and sch["after"] == (mode == "after")
        Y = torch.empty_like(Yr)
        for _ in range(2):
            Y.fill_(float("nan"))
            plan.mrdft_forward(xd, Y)
            torch.cuda.synchronize()
            assert torch.equal(Y, Yr), (mode, graph)
    assert _check_ragged(Yr, x, offs, orders, ref) <= FWD_TOL

def test_workload4_tuned_graph_full_size():
    """The 1000-signal ragged batch (m in 8..18) through the plan the benchmark
    times: tuned schedule and graph replay, so the levels above 16 run as pass
    chains forked onto side streams inside the capture.  Two replays, with
    eager work on the stream between them, equal an eager plan with the same
    schedule bit for bit; the longest signals and one signal of every order are
    compared with the oracle."""
    need_gpu()
    d = workloads.make(4)
    x, offs, orders = d["x"], d["offsets"], d["orders"]
    log("workload 4 tuned + graph: %d signals, %d samples" % (len(orders), offs[-1]))
    graphed = api.Plan(offsets=offs, dtype="c64", tune=True, graph=True)
    sch = graphed.schedule()
    log("  tuned schedule %s" % sch)
    eager = api.Plan(offsets=offs, dtype="c64")
    eager.set_schedule(sch["tile_log"], sch["grid"], sch["order"], sch["serial"], sch["after"])
    xd = to_dev(x)
    Yg = torch.empty(graphed.n_out, dtype=torch.complex64, device="cuda")
    Ye = torch.empty_like(Yg)
    eager.mrdft_forward(xd, Ye)
    for r in range(2):
        Yg.fill_(float("nan"))
        graphed.mrdft_forward(xd, Yg)                  # first call captures, the second replays
        junk = torch.randn(1 << 22, device="cuda") * 3.0   # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(Yg, Ye), "graph call %d differs from the eager plan" % r
        del junk
    oo = graphed.output_offsets()
    pick = set(int(j) for j in np.nonzero(orders == 18)[0][:3]) | set(int(j) for j in np.nonzero(orders == 17)[0][:2])
    for o in np.unique(orders):
        pick.add(int(np.nonzero(orders == o)[0][-1]))
    Yh = Yg.cpu().numpy()
    for j in sorted(pick):
        mj = int(orders[j])
        ref = oracle.forward(x[offs[j]:offs[j + 1]].astype(np.complex128))
        err = worst_level_err(Yh[oo[j]:oo[j + 1]].reshape(mj, 1 << mj), ref)
        assert err <= FWD_TOL, (j, mj, err)


# ---------------------------------------------------------------------------
# Level-range plans: only levels lo..hi are stored (compact layout).

def _levels_ref(x, lo, hi):
    ref = oracle.forward(x.astype(np.complex128))
    m = ref.shape[0]
    return ref[lo - 1:min(hi, m)]


@pytest.mark.parametrize("dtype,orders,lo,hi", [
    ("r32", [16, 16], 5, 9),            # inside the tile only
    ("r32", [16, 14, 12, 9], 11, 14),   # tile and rows pieces
    ("r32", [17, 13], 13, 17),          # pieces and a pass level
    ("c64", [16, 12, 10], 3, 13),       # complex tile and pieces
    ("c64", [17, 11, 14], 12, 17),      # pieces and a pass level only
    ("c64", [8, 13], 1, 4),             # register levels only
    ("c64", [16, 15, 9], 14, 16),       # upper pieces only: no tile job is launched
    ("r32", [16, 12, 5], 14, 16),       # the same for real input; two signals keep no level
    ("r32", [10, 11, 9, 9, 9, 13], 3, 10),   # short real signals in the complex launch (one multi tile of 9s)
])
def test_level_range_forward_and_adjoint(dtype, orders, lo, hi):
    need_gpu()
    log("levels %s %s [%d, %d]" % (dtype, orders, lo, hi))
    x, offs = _ragged(orders, 60 + lo, dtype=dtype)
    plan = api.Plan(offsets=offs, dtype=dtype, levels=(lo, hi))
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    plan.mrdft_forward(to_dev(x), Y)
    oo = plan.output_offsets()
    Yh = Y.cpu().numpy()
    rng = np.random.default_rng(lo * 31 + hi)
    gys = []
    for j, m in enumerate(orders):
        ref = _levels_ref(x[offs[j]:offs[j + 1]], lo, hi)
        got = Yh[oo[j]:oo[j + 1]].reshape(ref.shape)
        assert worst_level_err(got, ref) <= FWD_TOL if ref.size else got.size == 0
        gys.append(workloads.gaussian_complex(rng, ref.shape))
    # adjoint: gradients of the kept levels only (the others are zero)
    gy = np.concatenate([g.reshape(-1) for g in gys]).astype(np.complex64)
    gx = torch.empty(plan.n_in, dtype=torch.complex64 if dtype == "c64" else torch.float32, device="cuda")
    plan.mrdft_adjoint(to_dev(gy), gx)
    gxh = gx.cpu().numpy()
    for j, m in enumerate(orders):
        full = np.zeros((m, 1 << m), dtype=np.complex128)
        kept = gys[j]
        if kept.size:
            full[lo - 1:lo - 1 + kept.shape[0]] = kept
        ref = oracle.adjoint(full)
        if dtype == "r32":
            ref = ref.real
        got = gxh[offs[j]:offs[j + 1]]
        assert np.linalg.norm(got - ref) <= 1e-5 * max(np.linalg.norm(ref), 1e-30), (j, m)


def test_level_range_uniform_shape():
    need_gpu()
    x = torch.randn(3, 1 << 13, device="cuda")
    plan = api.Plan(m=13, batch=3, dtype="r32", levels=(4, 20))
    Y = plan.forward(x)
    assert Y.shape == (3, 10, 1 << 13)
    ref = oracle.forward(x[1].cpu().numpy().astype(np.complex128))
    assert worst_level_err(Y[1].cpu().numpy(), ref[3:]) <= FWD_TOL


@pytest.mark.parametrize("lo,hi", [(1, 28), (3, 9)])
def test_complex_small_signal_runs(lo, hi):
    """Signals below 2^11 share 2048-sample tiles in runs of equal order:
    runs longer than a tile holds (300 signals of 8 samples), runs that end
    mid-tile, single signals between runs, signals that keep no level
    (order below lo) and the same through the persistent form."""
    need_gpu()
    orders = [3] * 300 + [5, 5, 10, 10, 10, 2, 2, 2, 2, 2, 11, 4] + [1] * 7 + [9, 13, 8, 8, 6]
    x, offs = _ragged(orders, 49 + lo)
    plan = api.Plan(offsets=offs, dtype="c64", levels=(lo, hi))
    xd = to_dev(x)
    for grid in (0, 5):
        plan.set_schedule(11, grid, "tiles_first")
        Y = torch.full((plan.n_out,), float("nan"), dtype=torch.complex64, device="cuda")
        plan.mrdft_forward(xd, Y)
        oo = plan.output_offsets()
        Yh = Y.cpu().numpy()
        assert not np.isnan(Yh).any(), "output not fully written"
        worst = 0.0
        for j, m in enumerate(orders):
            ref = oracle.forward(x[offs[j]:offs[j + 1]].astype(np.complex128))[lo - 1:min(hi, m)]
            got = Yh[oo[j]:oo[j + 1]]
            assert got.size == ref.size, (j, m)
            if ref.size:
                worst = max(worst, worst_level_err(got.reshape(ref.shape), ref))
        log("  grid %d worst rel err %.3e" % (grid, worst))
        assert worst <= FWD_TOL
