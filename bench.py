#!/usr/bin/env python3
"""Benchmark of the fused batched MrDFT on one MI355X.

Workload: 64 real float32 signals of N = 2^16 samples (m = 16), each a sum of
8 random sinusoids plus noise (seeded, synthetic); output 64 x 16 x 65536
complex64.  One step = one forward MrDFT of the whole batch (all levels,
inputs resident in HBM).  The JSON line also reports forward+adjoint, the
plain per-level form (one torch.fft launch per level, each re-reading x),
the kernel roofline and the FP64 CPU oracle on the same signals.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
EXTRA_NAMES = ("workload3", "workload4", "workload2_half", "workload2d", "workload5")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the complex workloads reported beside the headline line")
    ap.add_argument("--extra", default=",".join(EXTRA_NAMES),
                    help="comma-separated subset of the workloads beside the headline (%s)" % ",".join(EXTRA_NAMES))
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


def cpu_baseline(x_np, seconds):
    """The FP64 oracle as it stands (single thread), on whole signals of the
    same workload until `seconds` of CPU time have been spent."""
    import numpy as np
    import oracle
    n_sig = x_np.shape[0]
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.forward(x_np[done % n_sig].astype(np.complex128))
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    samples = done * x_np.shape[1]
    return {"value": samples / el / 1e9, "unit": "Gsamples/s", "cores": 1, "kind": "oracle",
            "sample": "%d whole signals (2^16 samples, all 16 levels) of the same workload in %.1f s, "
                      "single-threaded FP64 C oracle (recursive radix-2 FFT per window)" % (done, el)}


# Kernel sources whose rocprofv3 byte counters are recorded under profiles/.
TRAFFIC_SOURCES = {
    "fused_fwd": ("profiles/fused_fwd_r32_b64_m16.md",
                  ["mrdft_fwd_real.hip", "mrdft_tile_real.h", "mrdft_rows_real.h", "mrdft_device.h",
                   "mrdft_lds_fft.h", "mrdft_internal.h", "mrdft_api.hip"]),   # the job table sets the L2 reuse
}


def measured_traffic(kind):
    """HBM bytes per launch of `kind` (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed profile, or None when the kernel sources have changed
    since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    if kind not in TRAFFIC_SOURCES:
        return None
    prof, srcs = TRAFFIC_SOURCES[kind]
    h = hashlib.sha256()
    for f in sorted(srcs):
        with open(os.path.join(here, "paper_1507_02525_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        lines = open(os.path.join(here, prof)).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        parts = ln.strip().strip("`").split()
        if len(parts) == 5 and parts[0] == "traffic" and parts[1] == kind:
            kv = dict(p.split("=") for p in parts[2:])
            if kv["sources"] != h.hexdigest()[:16]:
                return None
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def extra_workloads(steps, warmup, HBM, names=EXTRA_NAMES):
    """Workloads beside the headline: one long complex signal (N = 2^24) and a
    ragged batch of 1000 complex signals (m in 8..18) through a tuned plan with
    graph replay (forward only), the real batch with packed half-spectrum
    output, the 2-D separable transform of 4 real 1024 x 1024 images, and the
    spectral loss forward + backward on 32 real pairs of 2^18 samples.  Inputs
    resident in HBM."""
    import numpy as np
    import torch
    from paper_1507_02525_amd import api, workloads
    out = {}
    for k, name in ((3, "one complex64 signal, N=2^24 (m=24), tuned plan"),
                    (4, "1000 complex64 signals, m~U{8..18}, int64 offsets, tuned plan, graph replay")):
        if "workload%d" % k not in names:
            continue
        d = workloads.make(k)
        if k == 3:
            x = torch.from_numpy(d["x"]).cuda().view(-1)
            plan = api.Plan(m=d["m"], batch=d["batch"], dtype="c64", tune=True)
        else:
            x = torch.from_numpy(d["x"]).cuda()
            plan = api.Plan(offsets=d["offsets"], dtype="c64", tune=True, graph=True)
        Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
        fn = lambda: plan.mrdft_forward(x, Y)   # noqa: E731
        for _ in range(warmup):
            fn()
        ms = timed(fn, steps, torch.cuda.synchronize)
        n_in = int(plan.n_in)
        byts = n_in * 8 + plan.n_out * 8
        out["workload%d" % k] = {"workload": name, "ms_per_call": round(ms, 4),
                                 "Gsamples_per_s": round(n_in / (ms * 1e-3) / 1e9, 3),
                                 "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM, 4),
                                 "schedule": plan.schedule()}
        del Y, x, plan
        torch.cuda.empty_cache()
    # the real batch with packed half-spectrum output (half the output bytes)
    if "workload2_half" in names:
        d = workloads.make(2)
        x = torch.from_numpy(d["x"]).cuda().view(-1)
        plan = api.Plan(m=d["m"], batch=d["batch"], dtype="r32", half=True)
        Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
        fn = lambda: plan.mrdft_forward(x, Y)   # noqa: E731
        for _ in range(warmup):
            fn()
        ms = timed(fn, steps, torch.cuda.synchronize)
        byts = int(plan.n_in) * 4 + plan.n_out * 8
        out["workload2_half"] = {"workload": "64 real float32 signals, N=2^16 (m=16), packed half-spectrum output",
                                 "ms_per_call": round(ms, 4),
                                 "Gsamples_per_s": round(plan.n_in / (ms * 1e-3) / 1e9, 3),
                                 "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM, 4)}
        del Y, x, plan
        torch.cuda.empty_cache()
    # two-dimensional separable transform: 4 real images of 1024 x 1024, all 100 level pairs
    if "workload2d" in names:
        rng = np.random.default_rng(1515)
        x = torch.from_numpy(workloads.gaussian_real(rng, (4, 1024, 1024))).cuda()
        plan2 = api.Plan2D(10, 10, batch=4, dtype="r32")
        Y = torch.empty(plan2.n_out, dtype=torch.complex64, device="cuda")
        fn = lambda: plan2.mrdft_forward2d(x, Y)   # noqa: E731
        for _ in range(warmup):
            fn()
        ms = timed(fn, steps, torch.cuda.synchronize)
        byts = plan2.n_in * 4 + plan2.n_out * 8
        out["workload2d"] = {"workload": "2-D separable, 4 real float32 images 1024 x 1024, 100 level pairs",
                             "ms_per_call": round(ms, 4),
                             "Gsamples_per_s": round(plan2.n_in / (ms * 1e-3) / 1e9, 3),
                             "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM, 4)}
        del Y, x, plan2
        torch.cuda.empty_cache()
    # spectral loss, forward + backward: 32 real pairs of 2^18 samples
    if "workload5" in names:
        d = workloads.make(5)
        x = torch.from_numpy(d["x"]).cuda().requires_grad_(True)
        z = torch.from_numpy(d["z"]).cuda()

        def loss_step():
            x.grad = None
            api.spectral_loss(x, z).backward()

        for _ in range(warmup):
            loss_step()
        ms = timed(loss_step, steps, torch.cuda.synchronize)
        out["workload5"] = {"workload": "spectral loss forward + backward, 32 real float32 pairs, N=2^18 (m=18)",
                            "ms_per_call": round(ms, 4),
                            "Gsamples_per_s": round(x.numel() / (ms * 1e-3) / 1e9, 3)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this benchmark measures one GPU only (the transform shards by signal; "
              "multi-GPU runs are not part of it). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    names = [n for n in args.extra.split(",") if n]
    unknown = sorted(set(names) - set(EXTRA_NAMES))
    if unknown:
        print("bench.py: unknown workload(s) %s; choose from %s" % (unknown, ",".join(EXTRA_NAMES)), file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1507_02525_amd import api, workloads

    if args.copy_calibration:
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    d = workloads.make(2)
    B, m = d["batch"], d["m"]
    N = 1 << m
    x = torch.from_numpy(d["x"]).cuda()
    plan = api.Plan(m=m, batch=B, dtype="r32")
    Y = torch.empty(plan.n_out, dtype=torch.complex64, device="cuda")
    gx = torch.empty(plan.n_in, dtype=torch.float32, device="cuda")
    xf = x.view(-1)
    sync = torch.cuda.synchronize

    def fwd():
        plan.mrdft_forward(xf, Y)

    def fwd_bwd():
        plan.mrdft_forward(xf, Y)
        plan.mrdft_adjoint(Y, gx)

    for _ in range(args.warmup):
        fwd()
        fwd_bwd()
    sync()

    # --- timed region: exactly K forward steps --------------------------------------
    ms = timed(fwd, args.steps, sync)
    samples = B * N
    value = samples / (ms * 1e-3) / 1e9
    alg_bytes = samples * 4 + plan.n_out * 8
    frac_step = alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS

    # --- per-kernel durations (HIP events on the launch stream), same K steps ---------
    plan.set_profiling(True)
    plan.read_profile()
    ms_prof = timed(fwd, args.steps, sync)
    prof = plan.read_profile()
    plan.set_profiling(False)
    # algorithmic bytes of each kernel kind per step: x read once, its levels written once
    fused_levels = min(m, 16)                     # real input: tiles and levels 13..16 in one launch
    per_kind_bytes = {"fused_fwd": samples * 4 + fused_levels * samples * 8,
                      "pass_fwd": (m - fused_levels) * samples * 8}
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    tot_ms, launches = kinds[dom]
    launches_per_step = launches / args.steps
    if len(kinds) == 1 and launches_per_step == 1:
        # the step is this one launch: average over the K back-to-back launches
        # of the timed region (per-launch events would add their own overhead)
        avg_ms = ms
        timing = "HIP events around the K back-to-back launches of the timed region"
    else:
        avg_ms = tot_ms / launches
        timing = "HIP events around each launch, on its stream"
    bytes_per_launch = per_kind_bytes[dom] / launches_per_step
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom),
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "avg_launch_us": round(avg_ms * 1e3, 2), "timing": timing,
                "launches_per_step": launches_per_step,
                "kernel_share_of_step": round(tot_ms / args.steps / ms_prof, 3)}

    # --- forward + adjoint ------------------------------------------------------------
    ms_fb = timed(fwd_bwd, args.steps, sync)

    # --- plain per-level form: one torch.fft (rocFFT) launch per level -----------------
    Yp = torch.empty(m, B, N, dtype=torch.complex64, device="cuda")

    def plain():
        xc = x.to(torch.complex64)
        for i in range(1, m + 1):
            torch.fft.fft(xc.view(B, N >> i, 1 << i), dim=-1, out=Yp[i - 1].view(B, N >> i, 1 << i))

    for _ in range(args.warmup):
        plain()
    ms_plain = timed(plain, args.steps, sync)

    # --- sampled parity of the timed output (signal 0, all levels) ---------------------
    rel = None
    try:
        import oracle
        fwd()
        sync()
        ref = oracle.forward(d["x"][0].astype(np.complex128))
        got = Y[: m * N].view(m, N).cpu().numpy().astype(np.complex128)
        rel = max(float(np.linalg.norm(got[i] - ref[i]) / np.linalg.norm(ref[i])) for i in range(m))
    except Exception as exc:  # the oracle is optional here; report why it is missing
        rel = "unavailable: %s" % exc

    # --- attainable HBM rates on this machine (context for the roofline fraction) -------
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
    attainable["achieved_over_write"] = round(roofline["achieved"] / attainable["write_GBps"], 4)
    del big, big2
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d["x"], args.cpu_seconds)

    extra = None if args.no_extra else extra_workloads(max(5, args.steps // 4), 2, HBM_PEAK_GBS, names)

    out = {
        "metric": "MrDFT Gsamples/s & % HBM peak, fwd and fwd+bwd, vs per-level form, rel err<=1e-6",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 real float32 signals, N=2^16 (m=16), sums of 8 random sinusoids + "
                               "0.1 N(0,1) noise; all 16 levels, complex64 output",
                   "batch": B, "m": m, "input": "r32", "output_bytes": plan.n_out * 8},
        "hbm_frac_step": round(frac_step, 4),
        "algorithmic_bytes_per_step": alg_bytes,
        "roofline": roofline,
        "attainable_hbm": attainable,
        "fwd_bwd": {"ms_per_step": round(ms_fb, 4), "value": round(samples / (ms_fb * 1e-3) / 1e9, 3),
                    "unit": "Gsamples/s",
                    "hbm_frac": round((2 * alg_bytes) / (ms_fb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "plain_per_level": {"ms_per_step": round(ms_plain, 4),
                            "value": round(samples / (ms_plain * 1e-3) / 1e9, 3),
                            "speedup_fused_vs_plain": round(ms_plain / ms, 3)},
        "rel_err_sampled": rel,
        "cpu_baseline": cpu,
        "profile_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kinds.items()},
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
