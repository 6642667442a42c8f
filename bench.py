#!/usr/bin/env python3
"""Throughput of the HRC hot path on one MI355X.

One step = one full forward solve (traced levels, merge up,
merge down, quadrant gather) of the 1024x1024 scene (128 disks, 256 opaque
boxes, 32 one-pixel sigma-100 lines, value-noise fog), inputs resident in HBM.
Prints one JSON line: Mpixel/s of fluence (value), plus the forward+backward
rate, the batched forward+backward rate against sequential single-scene calls,
the HBM roofline of the dominant kernel (HIP events recorded at each of its
launches' start and end) and the FP64
oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--only-forward", action="store_true",
                    help="time the forward only (for profiler runs)")
    ap.add_argument("--half-intervals", action="store_true",
                    help="with --only-forward: the 16-bit interval storage (for profiling)")
    ap.add_argument("--only-backward", action="store_true",
                    help="run hrc_backward only, --steps times (for profiler runs)")
    ap.add_argument("--kept", action="store_true",
                    help="with --only-backward: one forward keeping the pyramid, then the "
                         "backward reusing it (HRC_FLAG_KEEP_PYRAMID / _REUSE_PYRAMID)")
    return ap.parse_args()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    profile (scaled by the plain-copy calibration), or None when there is no
    such profile or the kernel source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hrc_merge_down_1024_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["source"])
    if rec["kernel"] != kernel or not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it), from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def adam_recovery(ctx, steps: int = 200, lr: float = 0.3, every: int = 10) -> dict:
    """The 256x256 differentiable workload: Adam on softplus-parameterised
    emission and attenuation from a uniform start (0.1, 0.1), loss = MSE between
    the fluence and the hidden scene's; the loss curve and the fields' RMSEs
    against the hidden scene (the fields are not identifiable from the fluence
    alone, so the loss is what falls)."""
    import numpy as np
    import torch
    from paper_2505_02041_amd import fluence
    from scenes import config4
    hidden = config4()
    dev = torch.device("cuda", 0)
    he = torch.from_numpy(hidden.eps).to(dev)
    hs = torch.from_numpy(hidden.sigma).to(dev)
    with torch.no_grad():
        Ft = fluence(he, hs)
    inv = float(np.log(np.expm1(0.1)))
    pe = torch.full(he.shape, inv, device=dev, requires_grad=True)
    ps = torch.full(he.shape, inv, device=dev, requires_grad=True)
    opt = torch.optim.Adam([pe, ps], lr=lr)
    curve = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        opt.zero_grad()
        loss = torch.mean((fluence(torch.nn.functional.softplus(pe),
                                   torch.nn.functional.softplus(ps)) - Ft) ** 2)
        loss.backward()
        opt.step()
        if i % every == 0 or i == steps - 1:
            curve.append([i, float(loss.detach())])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    with torch.no_grad():
        e = torch.nn.functional.softplus(pe)
        sg = torch.nn.functional.softplus(ps)
        rmse_e = float(torch.sqrt(torch.mean((e - he) ** 2)))
        rmse_s = float(torch.sqrt(torch.mean((sg - hs) ** 2)))
        e0 = float(torch.sqrt(torch.mean((0.1 - he) ** 2)))
        s0 = float(torch.sqrt(torch.mean((0.1 - hs) ** 2)))
    return {"steps": steps, "lr": lr, "loss_curve": curve,
            "loss_ratio_first_to_last": curve[0][1] / curve[-1][1],
            "rmse_emission": rmse_e, "rmse_emission_at_start": e0,
            "rmse_sigma_t": rmse_s, "rmse_sigma_t_at_start": s0,
            "ms_per_step": el / steps * 1e3}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method's "
              "multi-GPU sharding is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2505_02041_amd import Batch, Context
    from paper_2505_02041_amd import _lib
    from paper_2505_02041_amd.roofline import (HBM_PEAK_GBPS, backward_bytes, forward_bytes,
                                               forward_bytes_rgb, pass_bytes)
    from scenes import config2, config3, config5

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = Context(0)
    sc = config3()
    N = 10
    S = 1 << N
    eps = torch.from_numpy(sc.eps).to(dev)
    sig = torch.from_numpy(sc.sigma).to(dev)
    F = torch.empty_like(eps)
    rng = np.random.default_rng(0)
    dF = torch.from_numpy(rng.normal(size=(S, S)).astype(np.float32)).to(dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    if args.only_backward:
        if args.kept:
            res = ctx.reserve(N)
            ctx.hrc_forward(eps, sig, F, flags=_lib.HRC_FLAG_KEEP_PYRAMID, reserve=res)
            for _ in range(args.warmup + args.steps):
                ctx.hrc_backward(eps, sig, dF, flags=_lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
        else:
            for _ in range(args.warmup + args.steps):
                ctx.hrc_backward(eps, sig, dF)
        torch.cuda.synchronize()
        print(json.dumps({"backward_steps": args.steps, "kept": args.kept}))
        return

    # ---- forward: the metric ------------------------------------------------
    log(f"forward {S}x{S}: {args.warmup} warm-up, {args.steps} timed steps")
    fwd_flags = _lib.HRC_FLAG_HALF_INTERVALS if (args.half_intervals and args.only_forward) else 0
    fwd_s = timed(lambda: ctx.hrc_forward(eps, sig, F, flags=fwd_flags), args.steps, args.warmup)
    # ---- a plain device copy of 512 MB: the achievable-bandwidth reference ---
    nbytes = 512 << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    copy_s = timed(lambda: dst.copy_(src), 10, 2)
    del src, dst
    if args.only_forward:
        print(json.dumps({"ms_per_step": fwd_s * 1e3, "copy_GBps": 2 * nbytes / copy_s / 1e9}))
        return
    # ---- the method's error: the benchmark scene's fluence against a brute-force
    # FP64 ray march (4096 directions per pixel) on a 128x128 crop, stored by
    # tests/golden/make_bruteforce_crop.py ----------------------------------------
    accuracy = None
    bf_path = os.path.join(ROOT, "tests", "golden", "bruteforce_1024_crop.npz")
    if os.path.exists(bf_path):
        g = np.load(bf_path)
        r0, r1, c0, c1 = (int(v) for v in g["crop"])
        ctx.hrc_forward(eps, sig, F)
        Fc = F[r0:r1, c0:c1].double().cpu().numpy()
        bf = g["bruteforce"]
        rms = float(np.sqrt(np.mean((Fc - bf) ** 2)))
        rms_oracle = float(np.sqrt(np.mean((g["oracle_hrc"] - bf) ** 2)))
        accuracy = {"rmse_vs_bruteforce": rms, "relative_rmse": rms / float(np.sqrt(np.mean(bf ** 2))),
                    "oracle_hrc_rmse_vs_bruteforce": rms_oracle,
                    "crop": [r0, r1, c0, c1], "bruteforce_directions": int(g["directions"])}
    # ---- the forward at the other configurations' sizes (64^2, 256^2, 512^2:
    # the small and differentiable scenes; 2048^2, 4096^2 with the benchmark
    # scene's generator and feature counts: the method's time does not depend
    # on the scene) ------------------------------------------------------------
    from scenes import config1, config2, config4, scene_like_512
    fwd_by_size = {}
    for name, cfg in (("64", config1), ("256", config4), ("512", config2),
                      ("2048", lambda: scene_like_512(2048, 7, 128, 256)),
                      ("4096", lambda: scene_like_512(4096, 7, 128, 256))):
        c = cfg()
        e2 = torch.from_numpy(c.eps).to(dev)
        s2 = torch.from_numpy(c.sigma).to(dev)
        F2 = torch.empty_like(e2)
        t = timed(lambda: ctx.hrc_forward(e2, s2, F2), 20 if c.eps.shape[0] >= 2048 else 50, 3)
        fwd_by_size[name] = {"ms": t * 1e3, "mpixel_per_s": c.eps.size / t / 1e6}
        del e2, s2, F2
    ctx.release_workspaces()
    # ---- the cross blur of Eq. 21 after the gather (HRC_FLAG_BLUR) -----------
    fwd_blur_s = timed(lambda: ctx.hrc_forward(eps, sig, F, flags=_lib.HRC_FLAG_BLUR),
                       max(5, args.steps // 2), 2)
    # ---- with an environment map lighting the grid from outside --------------
    ctx.set_environment([1.0 + 0.5 * np.sin(2 * np.pi * k / 64) for k in range(64)])
    fwd_env_s = timed(lambda: ctx.hrc_forward(eps, sig, F), max(5, args.steps // 2), 2)
    ctx.set_environment(None)
    # ---- the paper's 16-bit interval storage (Section 5; HRC_FLAG_HALF_INTERVALS):
    # a separate, reduced-precision line, never the metric -----------------------
    Fh = torch.empty_like(eps)
    fwd_half_s = timed(lambda: ctx.hrc_forward(eps, sig, Fh, flags=_lib.HRC_FLAG_HALF_INTERVALS),
                       args.steps, 3)
    ctx.hrc_forward(eps, sig, F)
    big = F.abs() > 1e-3 * F.abs().max()
    half_dev = float(((Fh - F).abs() / F.abs().clamp_min(1e-30))[big].max())
    del Fh
    ctx.release_workspaces()
    # ---- six diffuse bounces (Section 4.2; Fig. 14 converges after 6) ---------
    alb = torch.full_like(eps, 0.5)
    fwd_6b_s = timed(lambda: ctx.hrc_multibounce_forward(eps, sig, alb, 6, out=F),
                     max(3, args.steps // 10), 1)
    # ---- three radiance channels over the benchmark scene's medium in one call
    # (hrc_forward_rgb: the channels share every transmittance) beside three
    # one-channel calls ------------------------------------------------------------
    eps3 = torch.stack([eps, torch.roll(eps, 37, 1), 0.3 * eps]).contiguous()
    F3 = torch.empty_like(eps3)
    rgb_s = timed(lambda: ctx.hrc_forward_rgb(eps3, sig, F3), args.steps, 3)
    rgb_half_s = timed(lambda: ctx.hrc_forward_rgb(eps3, sig, F3, flags=_lib.HRC_FLAG_HALF_INTERVALS),
                       args.steps, 3)
    # the RGB reverse (transmittance adjoints shared by the channels) beside
    # three one-channel reverses, plain and through the reserve space
    log("rgb forward+backward")
    g3 = torch.from_numpy(np.random.default_rng(3).normal(size=(3, S, S)).astype(np.float32)).to(dev)
    KP, RP = _lib.HRC_FLAG_KEEP_PYRAMID, _lib.HRC_FLAG_REUSE_PYRAMID
    rb_reps = max(5, args.steps // 5)
    rgb_bwd_s = timed(lambda: ctx.hrc_backward_rgb(eps3, sig, g3), rb_reps, 2)
    ch = [(eps3[c].contiguous(), g3[c].contiguous()) for c in range(3)]
    three_bwd_s = timed(lambda: [ctx.hrc_backward(e_, sig, g_) for e_, g_ in ch], rb_reps, 2)
    res3 = ctx.reserve_rgb(N)
    rgb_kept_s = timed(lambda: (ctx.hrc_forward_rgb(eps3, sig, F3, flags=KP, reserve=res3),
                                ctx.hrc_backward_rgb(eps3, sig, g3, flags=RP, reserve=res3)),
                       rb_reps, 2)
    reserve3_bytes = res3.numel()
    del res3
    res1 = ctx.reserve(N)
    three_kept_s = timed(lambda: [(ctx.hrc_forward(e_, sig, F, flags=KP, reserve=res1),
                                   ctx.hrc_backward(e_, sig, g_, flags=RP, reserve=res1))
                                  for e_, g_ in ch], rb_reps, 2)
    del res1, ch, g3, eps3, F3
    ctx.release_workspaces()
    # ---- the allocation-free forward (hrc_forward_static: the library's own
    # device scratch) beside hrc_forward at 512^2, its largest grid -------------
    c2 = config2()
    e2 = torch.from_numpy(c2.eps).to(dev)
    s2 = torch.from_numpy(c2.sigma).to(dev)
    F2 = torch.empty_like(e2)
    static_s = timed(lambda: ctx.hrc_forward_static(e2, s2, F2), 50, 3)
    plain512_s = timed(lambda: ctx.hrc_forward(e2, s2, F2), 50, 3)
    del e2, s2, F2
    # ---- the 256^2 differentiable workload: 200 Adam steps -------------------
    log("adam 200 steps at 256x256")
    adam = adam_recovery(ctx)
    # ---- forward + backward (the backward recomputes the forward) ------------
    log("forward+backward")
    fb_s = timed(lambda: (ctx.hrc_forward(eps, sig, F), ctx.hrc_backward(eps, sig, dF)),
                 max(5, args.steps // 2), 2)
    H = _lib.HRC_FLAG_HALF_INTERVALS
    fb_half_s = timed(lambda: (ctx.hrc_forward(eps, sig, F, flags=H),
                               ctx.hrc_backward(eps, sig, dF, flags=H)),
                      max(5, args.steps // 2), 2)
    # the forward keeps what the reverse reads in a reserve space, the
    # backward reads it instead of recomputing it
    K, R = _lib.HRC_FLAG_KEEP_PYRAMID, _lib.HRC_FLAG_REUSE_PYRAMID
    log("forward (kept) + backward (reused)")
    res = ctx.reserve(N)
    fb_kept_s = timed(lambda: (ctx.hrc_forward(eps, sig, F, flags=K, reserve=res),
                               ctx.hrc_backward(eps, sig, dF, flags=R, reserve=res)),
                      max(5, args.steps // 2), 2)
    fwd_kept_s = timed(lambda: ctx.hrc_forward(eps, sig, F, flags=K, reserve=res),
                       max(5, args.steps // 2), 2)
    reserve_bytes = res.numel()
    del res
    ctx.release_workspaces()

    # ---- per-pass kernel durations: the same launches as hrc_forward, each
    # with HIP events the runtime records at the kernel's own start and end ---
    log("per-pass kernel timing")
    per = {}
    reps = max(5, args.steps // 2)
    for _ in range(reps):
        for name, n, ms in ctx.hrc_profile_solve(eps, sig):
            tot_ms, tot_b, cnt = per.get(name, (0.0, 0.0, 0))
            per[name] = (tot_ms + ms, tot_b + pass_bytes(name, N, n), cnt + 1)
    dom = max(per, key=lambda k: per[k][0])
    d_ms, d_b, d_cnt = per[dom]
    avg_launch_us = d_ms / d_cnt * 1e3
    bytes_per_launch = d_b / d_cnt
    achieved = bytes_per_launch / (avg_launch_us * 1e-6) / 1e9
    passes = {k: {"launches_per_step": v[2] // reps, "ms_per_step": v[0] / reps,
                  "GBps": v[1] / (v[0] * 1e-3) / 1e9} for k, v in per.items()}
    step_bytes = forward_bytes(N)
    kernel_name = _lib.PASS_KERNELS[_lib.PASS_NAMES.index(dom)]
    # ---- the same for hrc_backward (the recomputed forward, then the reverse):
    # per pass, kernel time and algorithmic bytes over that time ---------------
    log("per-pass kernel timing of the backward")
    bper = {}
    breps = max(3, args.steps // 10)
    for _ in range(breps):
        for name, n, ms in ctx.hrc_profile_solve(eps, sig, dF):
            # the backward's traced-levels pass stores all three levels
            nb = pass_bytes("seed_all" if name == "seed" else name, N, n)
            tot_ms, tot_b, cnt = bper.get(name, (0.0, 0.0, 0))
            bper[name] = (tot_ms + ms, tot_b + nb, cnt + 1)
    backward_passes = {k: {"launches_per_call": v[2] // breps, "ms_per_call": v[0] / breps,
                           "us_per_launch": v[0] / v[2] * 1e3,
                           "GBps": v[1] / (v[0] * 1e-3) / 1e9,
                           "frac_of_hbm_peak": v[1] / (v[0] * 1e-3) / 1e9 / HBM_PEAK_GBPS}
                       for k, v in bper.items()}
    # ---- the same forward replayed from a HIP graph (ten solves captured in
    # one graph): the time between the passes is the GPU's drain and ramp at
    # each kernel boundary, which a graph keeps ---------------------------------
    log("graph replay of the forward")

    def graph_replay():
        ctx.hrc_forward(eps, sig, F)  # the workspace exists before the capture
        torch.cuda.synchronize()
        F_ref = F.clone()
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream(dev)
        cap.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(cap):
            ctx.hrc_forward(eps, sig, F)  # the capture stream's own cached workspace
            cap.synchronize()
            with torch.cuda.graph(graph, stream=cap):
                for _ in range(10):
                    ctx.hrc_forward(eps, sig, F)
        torch.cuda.current_stream(dev).wait_stream(cap)
        t = timed(graph.replay, max(3, args.steps // 10), 2) / 10
        torch.cuda.synchronize()
        return t, bool(torch.equal(F, F_ref))
    try:
        graph_s, graph_bitwise = graph_replay()
        graph_err = None
    except Exception as ex:  # reported, not fatal: the metric does not depend on it
        graph_s, graph_bitwise, graph_err = None, False, str(ex)[:200]
    kernel_sum_ms = sum(v["ms_per_step"] for v in passes.values())
    traffic = measured_traffic(kernel_name)

    out = {
        "metric": "Mpixel/s fluence fwd at 1024^2 (fwd+bwd, ms/frame and HBM roofline alongside)",
        "value": S * S / fwd_s / 1e6,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fwd_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": "hrc_forward 1024x1024, 1 channel: 128 disks, 256 opaque boxes, "
                               "32 thin sigma-100 lines, value-noise fog (seed 3)",
                   "grid": S, "quadrants": 4, "traced_levels": 3, "parallelism": "single GPU"},
        "accuracy_1024_crop": accuracy,
        "fwd_by_size": fwd_by_size,
        "fwd_blur_ms": fwd_blur_s * 1e3,
        "blur_overhead_us": (fwd_blur_s - fwd_s) * 1e6,
        "fwd_environment_ms": fwd_env_s * 1e3,
        "fwd_6_bounces_ms": fwd_6b_s * 1e3,
        "fwd_half_intervals": {
            "ms": fwd_half_s * 1e3, "mpixel_per_s": S * S / fwd_half_s / 1e6,
            "model_GBps": forward_bytes(N, 4) / fwd_half_s / 1e9,
            "max_rel_dev_vs_f32": half_dev,
            "bound": N * 2.0 ** -11,
            "note": "intervals stored as 16-bit halves (Section 5); reduced precision, not the metric"},
        "fwd_rgb": {"ms": rgb_s * 1e3, "ms_per_channel": rgb_s * 1e3 / 3,
                    "mpixel_per_s": S * S / rgb_s / 1e6,
                    "model_bytes_per_channel": forward_bytes_rgb(N) / 3,
                    "one_channel_model_bytes": step_bytes,
                    "model_GBps": forward_bytes_rgb(N) / rgb_s / 1e9,
                    "speedup_vs_three_calls": 3 * fwd_s / rgb_s,
                    "backward": {"ms": rgb_bwd_s * 1e3, "three_one_channel_ms": three_bwd_s * 1e3,
                                 "speedup_vs_three": three_bwd_s / rgb_bwd_s,
                                 "fwd_bwd_kept_ms": rgb_kept_s * 1e3,
                                 "three_one_channel_fwd_bwd_kept_ms": three_kept_s * 1e3,
                                 "reserve_GB": reserve3_bytes / 1e9,
                                 "note": "hrc_backward_rgb (adjoint intervals (dL_r, dL_g, dL_b, dT): "
                                         "the medium's adjoints shared) beside three hrc_backward calls; "
                                         "and the reserve-space pairs (kept forward, reused reverse)"},
                    "half_intervals": {"ms": rgb_half_s * 1e3, "ms_per_channel": rgb_half_s * 1e3 / 3,
                                       "model_bytes_per_channel": forward_bytes_rgb(N, 8) / 3,
                                       "model_GBps": forward_bytes_rgb(N, 8) / rgb_half_s / 1e9,
                                       "note": "the paper's storage: 16-bit RGB intervals; "
                                               "reduced precision, not the metric"},
                    "note": "three emission channels over the 1024x1024 scene's attenuation in "
                            "one hrc_forward_rgb call (16-byte intervals, transmittance shared)"},
        "fwd_static_512": {"ms": static_s * 1e3, "hrc_forward_ms": plain512_s * 1e3,
                           "note": "hrc_forward_static (no workspace argument, static device "
                                   "scratch) and hrc_forward on the 512x512 scene"},
        "adam_256": adam,
        "fwd_bwd_half_intervals": {"ms": fb_half_s * 1e3, "mpixel_per_s": S * S / fb_half_s / 1e6,
                                   "note": "forward and backward with 16-bit intervals (the "
                                           "reverse's adjoints stay FP32); reduced precision, "
                                           "not the metric"},
        "fwd_bwd_mpixel_per_s": S * S / fb_s / 1e6,
        "fwd_bwd_ms": fb_s * 1e3,
        "fwd_bwd_kept": {"ms": fb_kept_s * 1e3, "mpixel_per_s": S * S / fb_kept_s / 1e6,
                         "forward_ms": fwd_kept_s * 1e3, "reserve_GB": reserve_bytes / 1e9,
                         "note": "hrc_forward keeping the pyramid and cascade levels in a reserve "
                                 "space (HRC_FLAG_KEEP_PYRAMID), hrc_backward reading them "
                                 "(HRC_FLAG_REUSE_PYRAMID) instead of recomputing them; results "
                                 "bitwise those of fwd_bwd_ms's plain calls"},
        "fwd_model_GBps": step_bytes / fwd_s / 1e9,
        "fwd_model_frac_of_peak": step_bytes / fwd_s / 1e9 / HBM_PEAK_GBPS,
        "fwd_bwd_model_GBps": (step_bytes + backward_bytes(N)) / fb_s / 1e9,
        "copy_GBps": 2 * nbytes / copy_s / 1e9,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "avg_launch_us": avg_launch_us,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
        "passes": passes,
        "backward_passes": backward_passes,
        "graph_replay": {"ms_per_forward": graph_s * 1e3 if graph_s else None,
                         "direct_ms": fwd_s * 1e3,
                         "kernel_sum_ms": kernel_sum_ms, "bitwise_equal": graph_bitwise,
                         "error": graph_err,
                         "note": "ten hrc_forward calls captured in one HIP graph and replayed, "
                                 "beside the direct calls and the sum of the passes' kernel "
                                 "times: the gaps are the GPU's own, at each kernel boundary"},
        "paper_context_ms": {"512": 1.85, "1024": 7.67, "hardware": "RTX 3080 Laptop, fp16 RGB"},
    }

    # ---- batched forward+backward -------------------------------------------
    if not args.no_batch:
        log(f"batch: {args.batch_scenes} scenes, planning (autotune + graph capture)")
        scenes = config5(count=args.batch_scenes)
        items = []
        for i, s_ in enumerate(scenes):
            Ss = s_.eps.shape[0]
            g = np.random.default_rng(7000 + i).normal(size=(Ss, Ss)).astype(np.float32)
            items.append({"emission": torch.from_numpy(s_.eps).to(dev),
                          "sigma_t": torch.from_numpy(s_.sigma).to(dev),
                          "fluence": torch.empty((Ss, Ss), device=dev),
                          "grad_fluence": torch.from_numpy(g).to(dev),
                          "grad_emission": torch.empty((Ss, Ss), device=dev),
                          "grad_sigma_t": torch.empty((Ss, Ss), device=dev)})
        px = sum(it["emission"].numel() for it in items)
        t0 = time.perf_counter()
        b = Batch(items, ctx)
        plan_s = time.perf_counter() - t0
        log(f"batch planned in {plan_s:.1f} s; timing")
        bsteps = max(3, args.steps // 10)
        batch_s = timed(b.launch, bsteps, 1)
        b.status()

        def sequential():
            for it in items:
                ctx.hrc_forward(it["emission"], it["sigma_t"], it["fluence"])
                ctx.hrc_backward(it["emission"], it["sigma_t"], it["grad_fluence"])
        seq_s = timed(sequential, bsteps, 1)
        reserves = {}

        def sequential_kept():
            K, R = _lib.HRC_FLAG_KEEP_PYRAMID, _lib.HRC_FLAG_REUSE_PYRAMID
            for it in items:
                n_ = it["emission"].shape[0].bit_length() - 1
                if n_ not in reserves:
                    reserves[n_] = ctx.reserve(n_)
                ctx.hrc_forward(it["emission"], it["sigma_t"], it["fluence"], flags=K,
                                reserve=reserves[n_])
                ctx.hrc_backward(it["emission"], it["sigma_t"], it["grad_fluence"], flags=R,
                                 reserve=reserves[n_])
        seq_kept_s = timed(sequential_kept, bsteps, 1)
        reserves.clear()
        out["batch"] = {"scenes": len(items), "megapixels": px / 1e6,
                        "fwd_bwd_ms": batch_s * 1e3,
                        "fwd_bwd_mpixel_per_s": px / batch_s / 1e6,
                        "sequential_fwd_bwd_ms": seq_s * 1e3,
                        "sequential_mpixel_per_s": px / seq_s / 1e6,
                        "speedup_vs_sequential": seq_s / batch_s,
                        "sequential_kept_fwd_bwd_ms": seq_kept_s * 1e3,
                        "speedup_vs_sequential_kept": seq_kept_s / batch_s,
                        "plan_s": plan_s, "workspace_GB": b.workspace_bytes / 1e9,
                        "autotuned": b.describe(),
                        "candidates_fastest": sorted(b.candidates(), key=lambda c: c["ms"])[:8]}
        del b
        # every scene inside the one persistent kernel (HRC_FLAG_BATCH_PERSISTENT):
        # the launch shape the planner's split is measured against
        log("batch with every scene in the persistent kernel")
        bp = Batch(items, ctx, flags=_lib.HRC_FLAG_BATCH_PERSISTENT)
        bp_s = timed(bp.launch, bsteps, 1)
        bp.status()
        out["batch"]["persistent_only"] = {"fwd_bwd_ms": bp_s * 1e3,
                                           "speedup_vs_sequential": seq_s / bp_s,
                                           "speedup_vs_sequential_kept": seq_kept_s / bp_s,
                                           "workspace_GB": bp.workspace_bytes / 1e9,
                                           "autotuned": bp.describe()}
        del bp, items
        ctx.release_workspaces()

    # ---- the oracle on the host (reported baseline) ---------------------------
    if not args.no_cpu:
        from oracle import hrc as oracle
        log(f"oracle CPU baseline (~{args.cpu_seconds:.0f} s)")
        frames = 0
        t0 = time.perf_counter()
        while True:
            oracle.fluence(sc.eps, sc.sigma)
            frames += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": frames * S * S / el / 1e6, "unit": "Mpixel/s",
                               "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"{frames} full 1024x1024 forward frames of the same "
                                         f"scene, FP64 NumPy, single thread, {el:.1f} s",
                               "host_cpus": os.cpu_count()}
        # the oracle on the smaller configurations too (median of 3 frames)
        from scenes import config1, config2, config4
        by_size = {}
        for name, cfg in (("64x64", config1), ("256x256", config4), ("512x512", config2)):
            c = cfg()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                oracle.fluence(c.eps, c.sigma)
                ts.append(time.perf_counter() - t0)
            by_size[name] = sorted(ts)[1] * 1e3
        out["cpu_baseline"]["ms_per_frame_by_size"] = by_size
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
