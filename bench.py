#!/usr/bin/env python3
"""Benchmark of the batched MrDFT on one MI355X.

Headline workload: a ragged batch of 1000 complex64 signals of lengths 2^m_j,
m_j uniform on {8, ..., 18} (seeded, synthetic; the largest workload that is
quoted), packed back to back with an int64 offsets array.  One step = one
forward MrDFT of the whole batch (every level of every signal) through a
tuned plan replayed from a HIP graph, inputs resident in HBM.

The JSON line also carries, for the headline and for every side workload
(64 real signals of 2^16 samples; one complex signal of 2^24 samples; the
spectral loss forward + backward on 32 real pairs of 2^18 samples; packed
half-spectrum output; the 2-D separable transform):
  * the roofline of the dominant kernel (algorithmic bytes or flops per launch
    over its measured launch duration, HIP events on its stream),
  * a sampled parity figure of the timed output against the FP64 oracle,
  * the plain per-level forms on the same GPU (one torch.fft launch per level,
    each re-reading x; and this library's own one-level transform, one launch
    per level) with their time and byte ratios,
and the FP64 C oracle timed on the host (one core and all cores).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extra | --extra a,b] [--no-plain] [--tune-cache PATH]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import platform
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
VALU_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (256 CUs at 2.4 GHz)
SIDE_NAMES = ("workload2", "workload3", "workload5", "workload2_half", "workload2d")
ROOT = os.path.dirname(os.path.abspath(__file__))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the all-core oracle run (0: min(16, CPUs))")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--extra", default=",".join(SIDE_NAMES),
                    help="comma-separated side workloads (%s)" % ",".join(SIDE_NAMES))
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-level comparators")
    ap.add_argument("--side-only", action="store_true",
                    help="profiling aid: run only the --extra side workloads (no headline, no CPU baseline) "
                         "and print their JSON object")
    ap.add_argument("--tune-cache", default="",
                    help="tuning cache file (MRDFT_TUNE_CACHE): a second run reuses the schedules")
    return ap.parse_args()


def timed(fn, steps, sync):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    sync()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    sync()
    return e0.elapsed_time(e1) / steps


# ---------------------------------------------------------------------------
# FP64 oracle on the host: one core, then all cores (worker processes forked
# before the GPU is touched; each runs the unchanged oracle on whole signals).

_CPU = {}


def _oracle_signal(j):
    import numpy as np
    import oracle
    x, off = _CPU["x"], _CPU["off"]
    oracle.forward(x[off[j]:off[j + 1]].astype(np.complex128))
    return int(off[j + 1] - off[j])


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(d, workers, metric_unit="Gsamples/s"):
    import numpy as np
    off = d["offsets"]
    _CPU["x"], _CPU["off"] = d["x"], off
    n = len(off) - 1
    order = sorted(range(n), key=lambda j: -(off[j + 1] - off[j]))       # longest first (balance)
    t0 = time.perf_counter()
    done = sum(_oracle_signal(j) for j in range(n))
    t1 = time.perf_counter() - t0
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        done_p = sum(pool.map(_oracle_signal, order, chunksize=1))
    tp = time.perf_counter() - t0
    assert done == done_p == int(off[-1])
    return {"value": done / tp / 1e9, "unit": metric_unit, "cores": workers, "kind": "oracle",
            "sample": "all %d signals of the workload (%d samples, every level), FP64 C oracle (direct sums "
                      "for windows up to 2^12, recursive radix-2 FFT per window above), once on one core "
                      "(%.2f s) and once over %d worker processes (%.2f s wall)" % (n, done, t1, workers, tp),
            "one_core": {"value": done / t1 / 1e9, "seconds": round(t1, 3)},
            "all_cores": {"value": done / tp / 1e9, "seconds": round(tp, 3), "workers": workers},
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}


# ---------------------------------------------------------------------------
# Committed HBM byte counters (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)

def measured_traffic(profile, key, sources):
    """Bytes per launch recorded in `profile` for `key`, or None when the
    kernel sources have changed since the counters were taken."""
    h = hashlib.sha256()
    for f in sorted(sources):
        with open(os.path.join(ROOT, "paper_1507_02525_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        lines = open(os.path.join(ROOT, profile)).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        parts = ln.strip().strip("`").split()
        if len(parts) == 5 and parts[0] == "traffic" and parts[1] == key:
            kv = dict(p.split("=") for p in parts[2:])
            if kv["sources"] != h.hexdigest()[:16]:
                return None
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


C64_SOURCES = ["mrdft_fwd_c64.hip", "mrdft_tile_c64.h", "mrdft_rows_c64.h", "mrdft_device.h", "mrdft_lds_fft.h",
               "mrdft_internal.h", "mrdft_api.hip", "mrdft_xlane.h"]
R32_SOURCES = ["mrdft_fwd_real.hip", "mrdft_tile_real.h", "mrdft_rows_real.h", "mrdft_device.h", "mrdft_lds_fft.h",
               "mrdft_internal.h", "mrdft_api.hip", "mrdft_xlane.h"]
TRAFFIC = {
    ("workload4", "fused_fwd"): ("profiles/fused_c64_ragged1000.md", "fused_c64_ragged", C64_SOURCES),
    ("workload2", "fused_fwd"): ("profiles/fused_fwd_r32_b64_m16.md", "fused_fwd", R32_SOURCES),
}


def level_outputs(orders, lo, hi, half=False):
    """Complex outputs of levels lo..hi over signals of the given orders."""
    tot = 0
    for m in orders:
        k = max(0, min(hi, m) - lo + 1)
        tot += k * ((1 << m) >> (1 if half else 0))
    return tot


def roofline_of(plan, fn, steps, sync, kind_bytes, traffic_key=None):
    """Profile `fn` (the plan's launches bracketed by HIP events on their
    streams), pick the kernel kind with the most time and price it against
    the HBM peak with its algorithmic bytes per step (kind_bytes)."""
    plan.set_profiling(True)
    plan.read_profile()
    ms_prof = timed(fn, steps, sync)
    prof = plan.read_profile()
    plan.set_profiling(False)
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    tot_ms, launches = kinds[dom]
    avg_ms = tot_ms / launches
    per_launch = kind_bytes.get(dom, 0) * steps / launches
    ach = per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if traffic_key and (traffic_key, dom) in TRAFFIC:
        traffic = measured_traffic(*TRAFFIC[(traffic_key, dom)])
    return {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(per_launch), "avg_launch_us": round(avg_ms * 1e3, 2),
            "launches_per_step": launches / steps, "kernel_share_of_step": round(tot_ms / steps / ms_prof, 3),
            "timing": "HIP events around each launch, on the stream it runs on",
            "kinds_ms_per_step": {k: round(v[0] / steps, 4) for k, v in kinds.items()}}


def worst_level(got, ref):
    import numpy as np
    w = 0.0
    for i in range(ref.shape[0]):
        nr = np.linalg.norm(ref[i])
        w = max(w, float(np.linalg.norm(got[i] - ref[i]) / nr) if nr > 0 else float(np.linalg.norm(got[i])))
    return w


# ---------------------------------------------------------------------------
# Plain per-level forms (comparators of Section 6's per-level FFT method)

def plain_torch_fft(groups, steps, warmup, sync):
    """One torch.fft (rocFFT) launch per level, each re-reading x.  groups:
    [(x2d view [count, N] complex64, m)], written to per-group buffers
    (no scatter into the plan's layout)."""
    import torch
    bufs = [torch.empty(m, xg.shape[0], xg.shape[1], dtype=torch.complex64, device=xg.device) for xg, m in groups]

    def run():
        for (xg, m), buf in zip(groups, bufs):
            c, N = xg.shape
            for i in range(1, m + 1):
                torch.fft.fft(xg.view(c, N >> i, 1 << i), dim=-1, out=buf[i - 1].view(c, N >> i, 1 << i))

    for _ in range(warmup):
        run()
    ms = timed(run, steps, sync)
    del bufs
    return ms


def plain_own_levels(make_plan, levels, x, steps, warmup, sync):
    """This library's transform restricted to one level (a level-range plan),
    one launch sequence per level, each re-reading x."""
    import torch
    plans = [make_plan((i, i)) for i in range(1, levels + 1)]
    outs = [torch.empty(p.n_out, dtype=torch.complex64, device=x.device) for p in plans]

    def run():
        for p, o in zip(plans, outs):
            p.mrdft_forward(x, o)

    for _ in range(warmup):
        run()
    ms = timed(run, steps, sync)
    for p in plans:
        p.close()
    return ms


def plain_entry(ms_fused, ms_torch, ms_own, samples, plain_bytes, fused_bytes):
    """Time and byte ratios of the plain per-level forms against the fused path
    (plain_bytes: x read once per level and every level written once)."""
    out = {"plain_algorithmic_bytes": int(plain_bytes),
           "byte_ratio_plain_over_fused": round(plain_bytes / fused_bytes, 3)}
    if ms_torch is not None:
        out["torch_fft_per_level"] = {"ms": round(ms_torch, 4), "Gsamples_per_s": round(samples / (ms_torch * 1e-3) / 1e9, 3),
                                      "speedup_fused": round(ms_torch / ms_fused, 3)}
    if ms_own is not None:
        out["own_one_level_kernels"] = {"ms": round(ms_own, 4),
                                        "Gsamples_per_s": round(samples / (ms_own * 1e-3) / 1e9, 3),
                                        "speedup_fused": round(ms_own / ms_fused, 3)}
    sp = [v["speedup_fused"] for v in out.values() if isinstance(v, dict)]
    if sp:
        out["fused_at_least_2x"] = bool(min(sp) >= 2.0)
    return out


# ---------------------------------------------------------------------------

def headline(args, sync):
    """Workload 4: 1000 ragged complex64 signals, tuned plan, graph replay."""
    import numpy as np
    import torch
    import oracle
    from paper_1507_02525_amd import api, workloads
    d = workloads.make(4)
    orders = [int(o) for o in d["orders"]]
    x = torch.from_numpy(d["x"]).cuda()
    plan = api.Plan(offsets=d["offsets"], dtype="c64", tune=True, graph=True)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    fwd = lambda: plan.mrdft_forward(x, Y)        # noqa: E731
    for _ in range(args.warmup):
        fwd()
    sync()
    # --- timed region: exactly K forward steps -----------------------------------------
    ms = timed(fwd, args.steps, sync)
    n_in = int(plan.n_in)
    alg = n_in * 8 + plan.n_out * 8
    value = n_in / (ms * 1e-3) / 1e9
    # --- dominant kernel (eager launches of the same schedule, events on their streams) --
    kind_bytes = {"fused_fwd": n_in * 8 + 8 * level_outputs(orders, 1, 16),
                  "pass_fwd": 8 * level_outputs(orders, 17, 99)}
    roof = roofline_of(plan, fwd, args.steps, sync, kind_bytes, "workload4")
    # --- sampled parity of the timed output ---------------------------------------------
    oo = plan.output_offsets()
    off = d["offsets"]
    ords = d["orders"]
    pick = set(int(j) for j in np.nonzero(ords == 18)[0][:2]) | {int(np.nonzero(ords == 17)[0][0])}
    for o in np.unique(ords):
        pick.add(int(np.nonzero(ords == o)[0][-1]))
    Yh = Y.cpu().numpy()
    worst = 0.0
    for j in sorted(pick):
        mj = int(ords[j])
        ref = oracle.forward(d["x"][off[j]:off[j + 1]].astype(np.complex128))
        worst = max(worst, worst_level(Yh[oo[j]:oo[j + 1]].reshape(mj, 1 << mj), ref))
    del Yh
    res = {"ms": ms, "value": value, "alg": alg, "samples": n_in, "roofline": roof, "schedule": plan.schedule(),
           "parity": {"worst_rel_l2_per_level": worst, "signals_checked": len(pick),
                      "sample": "2 signals of m = 18, 1 of m = 17 and the last signal of every order, every level, "
                                "against the FP64 oracle"}}
    if not args.no_plain:
        groups = []
        xs = x.view(-1)
        for o in sorted(set(orders)):
            idx = np.concatenate([np.arange(off[j], off[j + 1]) for j in range(len(orders)) if orders[j] == o])
            groups.append((xs[torch.from_numpy(idx).cuda()].view(-1, 1 << o), o))     # gathered once, untimed
        ms_t = plain_torch_fft(groups, max(3, args.steps // 4), 2, sync)
        del groups
        torch.cuda.empty_cache()
        ms_o = plain_own_levels(lambda lv: api.Plan(offsets=d["offsets"], dtype="c64", levels=lv), 18, x,
                                max(3, args.steps // 4), 2, sync)
        plain_bytes = 8 * sum(o * (1 << o) for o in orders) + 8 * plan.n_out      # x re-read per level
        res["plain"] = plain_entry(ms, ms_t, ms_o, n_in, plain_bytes, alg)
        res["plain"]["note"] = ("torch.fft per order group and level (signals of one order gathered into one "
                                "batch beforehand, untimed; outputs in per-group buffers); own: one level-range "
                                "plan per level 1..18")
    del Y, x, plan
    torch.cuda.empty_cache()
    return res, d


def side_workload2(args, sync, half=False):
    import numpy as np
    import torch
    import oracle
    from paper_1507_02525_amd import api, workloads
    d = workloads.make(2)
    B, m = d["batch"], d["m"]
    N = 1 << m
    x = torch.from_numpy(d["x"]).cuda().view(-1)
    plan = api.Plan(m=m, batch=B, dtype="r32", half=half)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    fwd = lambda: plan.mrdft_forward(x, Y)        # noqa: E731
    steps = max(5, args.steps)
    for _ in range(args.warmup):
        fwd()
    ms = timed(fwd, steps, sync)
    samples = B * N
    out_b = 8 * plan.n_out
    alg = samples * 4 + out_b
    kind_bytes = {"fused_fwd": alg}
    roof = roofline_of(plan, fwd, steps, sync, kind_bytes, None if half else "workload2")
    Yh = Y.view(B, m, N >> (1 if half else 0)).cpu().numpy()
    worst = 0.0
    for b in (0, 63):
        ref = oracle.forward_half(d["x"][b]) if half else oracle.forward(d["x"][b].astype(np.complex128))
        worst = max(worst, worst_level(Yh[b], ref))
    del Yh
    name = "64 real float32 signals, N=2^16 (m=16), sums of 8 random sinusoids + 0.1 N(0,1) noise"
    r = {"workload": name + ("; packed half-spectrum output" if half else "; all 16 levels, complex64 output"),
         "ms_per_call": round(ms, 4), "Gsamples_per_s": round(samples / (ms * 1e-3) / 1e9, 3),
         "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg,
         "roofline": roof,
         "parity": {"worst_rel_l2_per_level": worst, "sample": "signals 0 and 63, every level, FP64 oracle"}}
    if not half:
        gx = torch.empty(plan.n_in, dtype=torch.float32, device="cuda")
        fb = lambda: (plan.mrdft_forward(x, Y), plan.mrdft_adjoint(Y, gx))     # noqa: E731
        for _ in range(2):
            fb()
        ms_fb = timed(fb, steps, sync)
        r["fwd_adjoint"] = {"ms_per_call": round(ms_fb, 4), "Gsamples_per_s": round(samples / (ms_fb * 1e-3) / 1e9, 3),
                            "hbm_frac": round(2 * alg / (ms_fb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        gref = oracle.adjoint(Y[: m * N].view(m, N).cpu().numpy().astype(np.complex128)).real
        g0 = gx[:N].cpu().numpy().astype(np.float64)
        r["fwd_adjoint"]["parity_rel_l2_signal0"] = float(np.linalg.norm(g0 - gref) / np.linalg.norm(gref))
        if not args.no_plain:
            xc_src = torch.from_numpy(d["x"]).cuda()
            bufs = torch.empty(m, B, N, dtype=torch.complex64, device="cuda")

            def plain():
                xc = xc_src.to(torch.complex64)          # the cast is part of the plain form
                for i in range(1, m + 1):
                    torch.fft.fft(xc.view(B, N >> i, 1 << i), dim=-1, out=bufs[i - 1].view(B, N >> i, 1 << i))

            for _ in range(2):
                plain()
            ms_t = timed(plain, max(3, steps // 2), sync)
            del bufs
            ms_o = plain_own_levels(lambda lv: api.Plan(m=m, batch=B, dtype="r32", levels=lv), m, x,
                                    max(3, steps // 2), 2, sync)
            r["plain"] = plain_entry(ms, ms_t, ms_o, samples, m * samples * 4 + out_b, alg)
    del Y, x, plan
    torch.cuda.empty_cache()
    return r


def side_workload3(args, sync):
    import numpy as np
    import torch
    import oracle
    from paper_1507_02525_amd import api, workloads
    d = workloads.make(3)
    m = d["m"]
    N = 1 << m
    x = torch.from_numpy(d["x"]).cuda().view(-1)
    plan = api.Plan(m=m, batch=1, dtype="c64", tune=True)
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    fwd = lambda: plan.mrdft_forward(x, Y)        # noqa: E731
    steps = max(5, args.steps // 2)
    for _ in range(2):
        fwd()
    ms = timed(fwd, steps, sync)
    alg = N * 8 + plan.n_out * 8
    kind_bytes = {"fused_fwd": N * 8 + 8 * 16 * N, "pass_fwd": 8 * (m - 16) * N}
    roof = roofline_of(plan, fwd, steps, sync, kind_bytes)
    x128 = d["x"][0].astype(np.complex128)
    Yl = Y.view(m, N)
    worst = 0.0
    for i in (m, 17):
        worst = max(worst, worst_level(Yl[i - 1].cpu().numpy()[None], oracle.forward_level(x128, i, oracle.FFT)[None]))
    for i in (5, 11, 12, 16, 20):
        L = 1 << i
        for w in (0, (N >> i) - 1):
            ref = oracle.forward_level(x128[w * L:(w + 1) * L], i, oracle.FFT)
            worst = max(worst, worst_level(Yl[i - 1, w * L:(w + 1) * L].cpu().numpy()[None], ref[None]))
    r = {"workload": "one complex64 signal, N=2^24 (m=24), i.i.d. N(0,1) parts, tuned plan",
         "ms_per_call": round(ms, 4), "Gsamples_per_s": round(N / (ms * 1e-3) / 1e9, 3),
         "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg,
         "schedule": plan.schedule(), "roofline": roof,
         "parity": {"worst_rel_l2_per_level": worst,
                    "sample": "levels 24 and 17 in full, first and last window of levels 5, 11, 12, 16, 20"}}
    if not args.no_plain:
        ms_t = plain_torch_fft([(x.view(1, N), m)], max(3, steps // 2), 1, sync)
        ms_o = plain_own_levels(lambda lv: api.Plan(m=m, batch=1, dtype="c64", levels=lv), m, x,
                                max(3, steps // 2), 1, sync)
        r["plain"] = plain_entry(ms, ms_t, ms_o, N, m * N * 8 + 8 * plan.n_out, alg)
    del Y, Yl, x, plan
    torch.cuda.empty_cache()
    return r


def transform_flops(m):
    """Flops of one MrDFT of 2^m samples by the paper's counts (eqs. (6)-(7)):
    beta = m(m+3)2^(m-3) complex multiplications (6 flops) and 2 beta complex
    additions (2 flops)."""
    beta = m * (m + 3) * (1 << (m - 3))
    return 6 * beta + 2 * 2 * beta


def side_workload5(args, sync):
    import numpy as np
    import torch
    import oracle
    from paper_1507_02525_amd import api, workloads
    d = workloads.make(5)
    B, m = d["x"].shape[0], 18
    N = 1 << m
    x = torch.from_numpy(d["x"]).cuda().requires_grad_(True)
    z = torch.from_numpy(d["z"]).cuda()

    def step():
        x.grad = None
        api.spectral_loss(x, z).backward()

    steps = max(5, args.steps // 2)
    for _ in range(args.warmup):
        step()
    ms = timed(step, steps, sync)
    # four transforms per step: Y(x - z) and Y(z) forward, Y(x - z) again and
    # its adjoint backward
    flops = 4 * B * transform_flops(m)
    ach = flops / (ms * 1e-3) / 1e12
    io = 2 * B * N * 4 + B * N * 4
    g = x.grad.detach().cpu().numpy().astype(np.float64)
    xd, zd = d["x"].astype(np.float64), d["z"].astype(np.float64)
    closed = 2 * (xd - zd) / np.sum(zd ** 2, axis=1, keepdims=True)
    gerr = float(max(np.linalg.norm(g[b] - closed[b]) / np.linalg.norm(closed[b]) for b in range(B)))
    num_den, Lt = api.spectral_loss_terms(x.detach(), z)
    nd = num_den.cpu().numpy()
    terr = 0.0
    for b in (0, B - 1):
        ndr, _ = oracle.spectral_loss(d["x"][b], d["z"][b])
        terr = max(terr, float(np.max(np.abs(nd[b] / ndr - 1))))
    r = {"workload": "spectral loss forward + backward, 32 real float32 pairs (x, z), N=2^18 (m=18), N(0,1)",
         "ms_per_call": round(ms, 4), "Gsamples_per_s": round(B * N / (ms * 1e-3) / 1e9, 3),
         "roofline": {"bound": "alu", "kernel": "whole step", "achieved": round(ach, 3), "peak": VALU_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TFLOPS, 4), "traffic": None,
                      "algorithmic_flops_per_step": flops,
                      "note": "4 transforms of 32 signals at the paper's operation count; HBM in/out of the "
                              "step (x, z, gx) %d B = %.4f of 8 TB/s" % (io, io / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)},
         "parity": {"gradient_worst_rel_l2_vs_closed_form": gerr, "loss_terms_worst_rel_err": terr,
                    "sample": "gradient of all 32 signals against 2(x - z)/||z||^2; num/den of signals 0 and 31 "
                              "against the FP64 oracle"}}
    if not args.no_plain:
        xs = x.detach().clone().requires_grad_(True)

        def plain_loss():
            xs.grad = None
            xc = (xs - z).to(torch.complex64)
            zc = z.to(torch.complex64)
            L = 0.0
            for i in range(1, m + 1):
                a = torch.fft.fft(xc.view(B, N >> i, 1 << i), dim=-1)
                c = torch.fft.fft(zc.view(B, N >> i, 1 << i), dim=-1)
                L = L + (a.abs() ** 2).sum(dim=(1, 2)) / (c.abs() ** 2).sum(dim=(1, 2))
            (L.sum() / m).backward()

        for _ in range(2):
            plain_loss()
        ms_p = timed(plain_loss, max(3, steps // 2), sync)
        gp = xs.grad.detach().cpu().numpy().astype(np.float64)
        r["plain"] = {"torch_fft_per_level_autograd": {"ms": round(ms_p, 4), "speedup_fused": round(ms_p / ms, 3),
                                                       "gradient_worst_rel_l2_vs_closed_form": float(max(
                                                           np.linalg.norm(gp[b] - closed[b]) / np.linalg.norm(closed[b])
                                                           for b in range(B)))},
                      "fused_at_least_2x": bool(ms_p / ms >= 2.0),
                      "note": "loss written with one torch.fft per level for x - z and z, backward by autograd"}
    del x, z
    torch.cuda.empty_cache()
    return r


def side_workload2d(args, sync):
    import numpy as np
    import torch
    import oracle
    from paper_1507_02525_amd import api, workloads
    rng = np.random.default_rng(1515)
    xn = workloads.gaussian_real(rng, (4, 1024, 1024))
    x = torch.from_numpy(xn).cuda()
    plan2 = api.Plan2D(10, 10, batch=4, dtype="r32")
    Y = torch.empty(plan2.n_out, dtype=torch.complex64, device="cuda")
    fn = lambda: plan2.mrdft_forward2d(x, Y)      # noqa: E731
    steps = max(5, args.steps // 2)
    for _ in range(2):
        fn()
    ms = timed(fn, steps, sync)
    alg = plan2.n_in * 4 + plan2.n_out * 8
    # parity: level pairs of image 0 against the 2-D oracle on a 64 x 64 corner
    # block (every pair whose blocks fit inside it is exact on the corner)
    Yv = Y.view(4, 10, 1024, 10, 1024)
    ref = oracle.forward2d(xn[0, :64, :64].astype(np.float64))        # (6, 6, 64, 64)
    worst = 0.0
    for i1 in range(6):
        for i2 in range(6):
            got = Yv[0, i1, :64, i2, :64].cpu().numpy()
            worst = max(worst, worst_level(got.reshape(1, -1), ref[i1, i2].reshape(1, -1)))
    r = {"workload": "2-D separable, 4 real float32 images 1024 x 1024, 100 level pairs",
         "ms_per_call": round(ms, 4), "Gsamples_per_s": round(plan2.n_in / (ms * 1e-3) / 1e9, 3),
         "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "roofline": {"bound": "hbm", "kernel": "whole call (transposes + two 1-D transforms)",
                      "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                      "algorithmic_bytes_per_launch": alg},
         "parity": {"worst_rel_l2_per_level_pair": worst,
                    "sample": "image 0, level pairs (1..6, 1..6) on the 64 x 64 corner block, FP64 oracle"}}
    del Y, x, plan2
    torch.cuda.empty_cache()
    return r


SIDE_FN = {"workload2": lambda args, sync: side_workload2(args, sync),
           "workload2_half": lambda args, sync: side_workload2(args, sync, half=True),
           "workload3": side_workload3,
           "workload5": side_workload5,
           "workload2d": side_workload2d}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this benchmark measures one GPU only (the transform shards by signal; "
              "multi-GPU runs are not part of it). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    names = [] if args.no_extra else [n for n in args.extra.split(",") if n]
    unknown = sorted(set(names) - set(SIDE_NAMES))
    if unknown:
        print("bench.py: unknown workload(s) %s; choose from %s" % (unknown, ",".join(SIDE_NAMES)), file=sys.stderr)
        sys.exit(2)
    if args.tune_cache:
        os.environ["MRDFT_TUNE_CACHE"] = args.tune_cache
    sys.path.insert(0, ROOT)
    from paper_1507_02525_amd import workloads

    # the host oracle first: its worker processes are forked before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline and not args.side_only:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(workloads.make(4), workers)

    import torch
    sync = torch.cuda.synchronize
    if args.copy_calibration:
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        sync()
        del src, dst

    if args.side_only:
        side = {n: SIDE_FN[n](args, sync) for n in names}
        print(json.dumps({"side_only": True, "steps": args.steps, "side_workloads": side}), flush=True)
        return

    h, _ = headline(args, sync)

    # attainable HBM rates on this machine (context for the roofline fractions)
    big = torch.empty(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
    big2 = torch.empty_like(big)
    for _ in range(3):
        big.fill_(1.0)
        big2.copy_(big)
    ms_fill = timed(lambda: big.fill_(1.0), 10, sync)
    ms_copy = timed(lambda: big2.copy_(big), 10, sync)
    attainable = {"write_GBps": round(big.numel() * 4 / (ms_fill * 1e-3) / 1e9, 1),
                  "copy_GBps": round(2 * big.numel() * 4 / (ms_copy * 1e-3) / 1e9, 1),
                  "how": "torch fill_ (write) and copy_ (read + write) of 1 GiB, 3 warm-up and 10 timed reps"}
    attainable["step_over_write_rate"] = round(h["alg"] / (h["ms"] * 1e-3) / 1e9 / attainable["write_GBps"], 4)
    del big, big2
    torch.cuda.empty_cache()

    side = {n: SIDE_FN[n](args, sync) for n in names}

    out = {
        "metric": "MrDFT Gsamples/s & % HBM peak, fwd and fwd+bwd, vs per-level form, rel err<=1e-6",
        "value": round(h["value"], 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1000 complex64 signals of lengths 2^m, m uniform in [8, 18], i.i.d. N(0,1) parts, "
                               "packed with int64 offsets; every level of every signal; tuned plan, HIP graph replay",
                   "signals": 1000, "samples": h["samples"], "input": "c64", "schedule": h["schedule"]},
        "hbm_frac_step": round(h["alg"] / (h["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": h["alg"],
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "parity": h["parity"],
        "plain_per_level": h.get("plain"),
        "attainable_hbm": attainable,
        "side_workloads": side,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
