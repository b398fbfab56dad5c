"""Levels above 16 computed by global passes, against the FP64 oracle.

From level 18 up a level is built from the level below: the even bins are
the sums of the child windows' bins (Section 3, eq. (2)), the odd bins the
half-length DFT of the twiddled difference of the window's halves (eq. (3)),
both over global passes (levels 17 and 18 sharing their first and last
launches, which also take level 17 of the signals of order 17 when the
pass scratch holds it).  Covered: ragged complex and real batches; level
ranges that keep the level below (recurrence) or not (direct passes); every
stream schedule; graph replay against the eager plan bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import api, workloads
from tests.gpu_util import FWD_TOL, log, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _ragged(orders, seed, dtype):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum([1 << o for o in orders])]).astype(np.int64)
    n = int(offs[-1])
    x = workloads.gaussian_complex(rng, (n,)) if dtype == "c64" else workloads.gaussian_real(rng, (n,))
    return x, offs


def _check_upper(Yh, x, offs, orders, lo, hi, oo):
    """Levels max(lo, 17)..min(hi, m) of every signal in full; every stored
    value finite (the output was NaN-filled)."""
    assert np.all(np.isfinite(Yh)), "unwritten outputs"
    worst = 0.0
    for j, m in enumerate(orders):
        n = 1 << m
        kept = max(0, min(hi, m) - lo + 1)
        got = Yh[oo[j]:oo[j + 1]].reshape(kept, n) if kept else None
        seg = x[offs[j]:offs[j + 1]].astype(np.complex128)
        for i in range(max(lo, 17), min(hi, m) + 1):
            ref = oracle.forward_level(seg, i, oracle.FFT)
            err = rel_l2(got[i - lo], ref)
            assert err <= FWD_TOL, (j, m, i, err)
            worst = max(worst, err)
    return worst


@pytest.mark.parametrize("dtype,orders,lo,hi", [
    ("c64", [20, 19, 21], 1, 28),       # every level; three orders in one plan
    ("c64", [21, 20], 19, 21),          # level 19 by direct passes (18 not kept), 20 and 21 from the level below
    ("c64", [20], 20, 20),              # a single upper level: direct passes
    ("c64", [21, 19], 18, 20),          # 19 and 20 from the level below, 21 not kept
    ("c64", [19, 18], 17, 18),          # levels 17 and 18 only: their shared head and tail launches
    ("r32", [20, 19], 1, 28),           # real input (difference of real halves)
    # signals of order 17 run their level 17 inside the shared head and tail
    # launches of the first longer group when the scratch holds both
    ("c64", [17, 18, 17, 19], 1, 28),   # with the order-18 group's head and tail
    ("r32", [17, 19, 17], 1, 28),       # with an order-19 group's; the scratch exactly full
    ("c64", [17, 17, 17, 18], 1, 28),   # scratch too small: separate passes
    ("c64", [18, 17], 17, 18),          # levels 17 and 18 only
    ("c64", [18, 17], 17, 17),          # level 17 only: no shared launches
])
def test_upper_levels_every_schedule(dtype, orders, lo, hi):
    need_gpu()
    log("upper levels %s %s [%d, %d]" % (dtype, orders, lo, hi))
    x, offs = _ragged(orders, 1900 + 7 * lo + hi, dtype)
    plan = api.Plan(offsets=offs, dtype=dtype, levels=(lo, hi))
    sch = plan.schedule()
    xd = to_dev(x)
    oo = plan.output_offsets()
    first = None
    for serial, after in ((False, False), (True, False), (False, True)):
        plan.set_schedule(sch["tile_log"], sch["grid"], sch["order"], serial, after)
        Y = torch.full((plan.n_out,), float("nan"), dtype=torch.complex64, device="cuda")
        plan.mrdft_forward(xd, Y)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        if first is None:
            first = Yh
            worst = _check_upper(Yh, x, offs, orders, lo, hi, oo)
            log("  worst relative L2 of the upper levels %.2e" % worst)
        else:                                          # the schedule moves launches, not arithmetic
            assert np.array_equal(Yh, first), (serial, after)


def test_upper_levels_graph_replay():
    need_gpu()
    orders = [21, 20, 19]
    log("upper levels graph replay c64 %s" % orders)
    x, offs = _ragged(orders, 1999, "c64")
    xd = to_dev(x)
    eager = api.Plan(offsets=offs, dtype="c64")
    graphed = api.Plan(offsets=offs, dtype="c64", graph=True)
    Ye = torch.empty(eager.n_out, dtype=torch.complex64, device="cuda")
    eager.mrdft_forward(xd, Ye)
    for r in range(3):
        Yg = torch.full_like(Ye, float("nan"))
        graphed.mrdft_forward(xd, Yg)                  # the first call captures, the others replay
        junk = torch.randn(1 << 22, device="cuda") * 3.0
        torch.cuda.synchronize()
        assert torch.equal(Yg, Ye), "graph call %d differs from the eager plan" % r
        del junk
    _check_upper(Ye.cpu().numpy(), x, offs, orders, 1, 28, eager.output_offsets())


@pytest.mark.parametrize("seed", [6, 7, 4, 0])      # shared launches; scratch too small; real with an
def test_upper_levels_random_mixes(seed):              # order-19 partner only; level 17 the top kept level
    """Random ragged mixes of orders 16..19 (shuffled, 1..3 signals of each
    order present) and random level ranges: whether the signals of order 17
    ride in the shared launches depends on the mix and on the scratch size,
    so these cover both outcomes and the ranges that switch the shared
    launches off; every kept upper level against the oracle, every schedule
    bit for bit."""
    need_gpu()
    rng = np.random.default_rng(4200 + seed)
    orders = []
    for o in (16, 17, 18, 19):
        orders += [o] * int(rng.integers(0 if o != 17 else 1, 4))
    rng.shuffle(orders)
    dtype = "r32" if seed == 4 else "c64"
    lo = int(rng.choice([1, 12, 16, 17]))
    hi = int(rng.choice([17, 18, 28]))
    log("upper levels random mix %s %s [%d, %d]" % (dtype, orders, lo, hi))
    x, offs = _ragged(orders, 4300 + seed, dtype)
    plan = api.Plan(offsets=offs, dtype=dtype, levels=(lo, hi))
    sch = plan.schedule()
    xd = to_dev(x)
    oo = plan.output_offsets()
    first = None
    for serial, after in ((False, False), (True, False), (False, True)):
        plan.set_schedule(sch["tile_log"], sch["grid"], sch["order"], serial, after)
        Y = torch.full((plan.n_out,), float("nan"), dtype=torch.complex64, device="cuda")
        plan.mrdft_forward(xd, Y)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        if first is None:
            first = Yh
            worst = _check_upper(Yh, x, offs, orders, lo, hi, oo)
            log("  worst relative L2 of the upper levels %.2e" % worst)
        else:
            assert np.array_equal(Yh, first), (serial, after)
