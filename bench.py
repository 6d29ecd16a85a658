"""Encoder throughput of the Cool-chic rate-distortion pass on one MI355X.

One step = one training iteration at 768x512 (Section IV-A): forward, hand
written backward and Adam update of the latents and every decoder parameter,
all through the HIP library's C ABI.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload full|low]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encoder fwd+bwd iters/s @768x512 (% FP32 roofline)"
FP32_PEAK_TFLOPS = 157.3       # MI355X dense FP32 (vector and matrix)
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (arch tuple, description)
    "full": ((7, 24, 2, 8, 40, 2), "full768x512: 7 levels, ARM 24-24-24-2 on the 24 causal neighbours of a 7x7 "
                                   "window, separable 8-tap upsampling per level, synthesis 7-40-3 + 2 residual "
                                   "3x3 convs; 200-blob synthetic image; lambda 1e-3; Adam lr 1e-2"),
    "low": ((7, 8, 2, 8, 16, 1), "low768x512: 7 levels, ARM 8-8-8-2 on 8 causal neighbours, separable 8-tap "
                                 "upsampling per level, synthesis 7-16-3 + 1 residual 3x3 conv; 200-blob synthetic "
                                 "image; lambda 1e-3; Adam lr 1e-2"),
}


def algorithmic_counts(arch, H, W):
    """Per-iteration algorithmic work (Eq. (2): backward = 2x forward MAC)."""
    L, C, NH, K, Hs, R = arch
    n_lat = sum((H >> l) * (W >> l) for l in range(L))
    n_px = H * W
    arm_mac_per_latent = NH * C * C + 2 * C
    ups_outputs = sum((L - 1 - s) * (H >> s) * (W >> s) for s in range(L - 1))
    ups_mac = ups_outputs * (K / 4 + K / 2)
    syn_mac_per_px = L * Hs + Hs * 3 + R * 81
    fwd_mac = arm_mac_per_latent * n_lat + ups_mac + syn_mac_per_px * n_px
    return dict(n_lat=n_lat, n_px=n_px, arm_flop=6.0 * arm_mac_per_latent * n_lat,
                syn_flop=6.0 * syn_mac_per_px * n_px, iter_flop=6.0 * fwd_mac, kappa_dec=fwd_mac / n_px)


ARM_SOURCES = ("paper_2403_11651_amd/csrc/arm.hip", "paper_2403_11651_amd/csrc/common.hpp",
               "paper_2403_11651_amd/csrc/rate.hpp", "paper_2403_11651_amd/csrc/kernels.hpp")


def arm_traffic_from_profile(workload):
    """HBM bytes per ARM launch from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None if there is none for this workload or the kernel sources
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"arm_kernel_{workload}768x512.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ARM_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_inputs(arch, H=512, W=768):
    from paper_2403_11651_amd import workloads as WL
    L, C, NH, K, Hs, R = arch
    na = NH * (C * C + C) + 2 * C + 2
    nu = (L - 1) * 2 * K
    ns = Hs * L + Hs + 3 * Hs + 3 + R * 84
    img = WL.image(10, H, W, 200)
    y = WL.latents(11, H, W, L)
    w = WL.weights(12, na + nu + ns)
    return img, y, w[:na], w[na:na + nu], w[na + nu:]


BATCH_ARCH = (7, 8, 2, 8, 16, 1)
BATCH_DESC = ("32 images, sizes drawn uniformly from 256x256 .. 1024x768 in steps of 64 (seed 999), each with its "
              "own 7-level Laplace latent pyramid and its own low-complexity decoder (ARM 8-8-8-2, synthesis "
              "7-16-3 + 1 residual 3x3 conv); blob count 200 per 768x512 of area; lambda 1e-3; Adam lr 1e-2")


def batch_inputs(B, n=32):
    """The batched-overfitting workload: problems, images, initial latents and
    initial (arm, ups, syn) parameters of each image."""
    from paper_2403_11651_amd import workloads as WL
    L, C, NH, K, Hs, R = BATCH_ARCH
    na = NH * (C * C + C) + 2 * C + 2
    nu = (L - 1) * 2 * K
    ns = Hs * L + Hs + 3 * Hs + 3 + R * 84
    probs, images, y0, params0 = [], [], [], []
    for k, (H, W) in enumerate(WL.batch_sizes(999, n)):
        probs.append(B.Problem(H, W, B.Arch(*BATCH_ARCH), B.CC_QUANT_ROUND, 1e-3))
        images.append(WL.image(1000 + k, H, W, max(1, round(200 * H * W / (768 * 512)))))
        y0.append(WL.latents(2000 + k, H, W, L))
        w = WL.weights(3000 + k, na + nu + ns)
        params0.append((w[:na], w[na:na + nu], w[na + nu:]))
    return probs, images, y0, params0


def run_batched(B, iters, graph_steps=50, log=None):
    """Overfits the 32-image batch for `iters` iterations (autotuned launch
    shape, graph replays of graph_steps iterations); returns the record."""
    import torch
    from paper_2403_11651_amd import batch as BT
    if iters % graph_steps:
        raise ValueError("--batch-iters must be a multiple of the graph length")
    probs, images, y0, params0 = batch_inputs(B)
    enc = BT.BatchEncoder(probs, images, y0, params0)
    t0 = time.perf_counter()
    tuned = BT.autotune(enc, log=log)
    tune_s = time.perf_counter() - t0
    enc.backward()
    torch.cuda.synchronize()
    loss0 = enc.loss.cpu().numpy().copy()
    t0 = time.perf_counter()
    g = enc.capture(graph_steps)
    capture_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for r in range(iters // graph_steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1000.0
    enc.backward()  # the loss of the final parameters
    torch.cuda.synchronize()
    l4 = enc.loss.cpu().numpy()
    if np.any(l4[:, 3] != 0.0) or not np.all(np.isfinite(l4[:, 0])):
        raise RuntimeError(f"non-finite loss in the batched run: {l4}")
    px = sum(p.H * p.W for p in probs)
    return {"workload": BATCH_DESC, "images": len(probs), "pixels": px, "iterations": iters,
            "seconds": round(secs, 4), "images_per_s": round(len(probs) / secs, 4),
            "ms_per_iteration": round(1000.0 * secs / iters, 5),
            "mpix_iters_per_s": round(px * iters / secs / 1e6, 1),
            "tuning": {"arm_blocks": tuned["tune"][0], "syn_blocks": tuned["tune"][1], "cached": tuned["cached"],
                       "tune_s": round(tune_s, 2), "candidates_ms": tuned.get("timings")},
            "graph_steps": graph_steps, "capture_s": round(capture_s, 4),
            "loss_start_mean": float(loss0[:, 0].mean()), "loss_end_mean": float(l4[:, 0].mean()),
            "psnr_end_mean_db": float(np.mean(10.0 * np.log10(1.0 / l4[:, 1]))),
            "rate_end_bpp_mean": float(np.mean(l4[:, 2] / np.array([p.H * p.W for p in probs])))}


WARM_TRAIN, WARM_HELD, WARM_ITERS = 256, 32, 500


def warm_start_images():
    """Images of the bounded warm-start run, generated in worker processes
    (before this process touches the GPU)."""
    from paper_2403_11651_amd import warmstart_eval as WE
    return (WE.make_images([10000 + i for i in range(WARM_TRAIN)], 512, 768),
            WE.make_images([20000 + i for i in range(WARM_HELD)], 512, 768))


def run_warm_start(images, iters=WARM_ITERS, log=None):
    """A bounded run of the warm-start experiment at 768x512 (pairs from the
    plain encoder, regression then rate-distortion training of the network,
    held-out evaluation); returns the seconds per image to the plain
    encoder's result with and without the warm start."""
    from paper_2403_11651_amd import warmstart_eval as WE
    tr, ho = images
    n_train, n_held = len(tr), len(ho)
    res = WE.run(tr, ho, iters, epochs=40, rd_epochs=20, schedules=((30, 2e-3),), log=log)
    r = res["heldout_results"]
    warm = r["rd_round_noise30_lr0.002"]
    return {"workload": f"{n_train} training pairs and {n_held} held-out 768x512 images (seeds 10000 + i, "
                        f"20000 + i), low-complexity decoder, plain encoder {iters} iterations (80 % noise proxy, "
                        f"then rounding)",
            "s_per_image_plain": round(r["plain"]["s_per_image"], 5),
            "s_per_image_warm": round(warm["s_per_image"], 5),
            "speedup": round(r["plain"]["s_per_image"] / warm["s_per_image"], 3),
            "criterion_met": warm["criterion_met"], "met_at_start": warm["met_at_start"],
            "fallbacks": warm["fallbacks"], "iters_median": warm["iters_median_criterion"],
            "plain_psnr_db": round(r["plain"]["psnr_mean"], 3), "plain_bpp": round(r["plain"]["bpp_mean"], 4),
            "untrained_criterion_met": r["untrained_noise30_lr0.002"]["criterion_met"],
            "pair_generation_s": res["pair_generation_s"], "train_s": res["train_s"],
            "rd_train_s": res["rd_round_train_s"]}


def cpu_baseline(arch, budget_s=20.0):
    """The FP64 oracle, single-threaded, timed on full 768x512 iterations
    (forward + backward + Adam) until about budget_s seconds have passed."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import oracle as O
    img, y, arm, ups, syn = make_inputs(arch)
    A = O.Arch(*arch)
    theta = np.concatenate([y, arm, ups, syn]).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    na, nu = arm.size, ups.size
    ny = y.size
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    n = 0
    t0 = time.perf_counter()
    try:
        while True:
            yy, aa = theta[:ny], theta[ny:ny + na]
            uu, ss = theta[ny + na:ny + na + nu], theta[ny + na + nu:]
            out = O.backward(A, img, yy, aa, uu, ss, 1e-3)
            g = np.concatenate([out["g_y"], out["g_arm"], out["g_ups"], out["g_syn"]])
            theta, m, v = O.adam_step(theta, g, m, v, n + 1)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="iters/s", cores=1, kind="oracle",
                sample=f"{n} full iterations (forward + backward + Adam) of the same 768x512 workload in FP64, "
                       f"{dt:.1f} s, one thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--batch-iters", type=int, default=2000,
                    help="iterations of the 32-image batched overfitting run (0 skips it)")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the bounded warm-start experiment")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (a known-size reference for "
                         "the FETCH_SIZE / WRITE_SIZE hardware counters); not part of any timed step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path runs one image per GPU and images shard across GPUs with no "
              f"communication, so --gpus {args.gpus} is not run here", file=sys.stderr)
        sys.exit(2)

    warm_images = None if args.no_warm_start else warm_start_images()
    import torch
    from paper_2403_11651_amd import binding as B
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    arch, desc = WORKLOADS[args.workload]
    H, W = 512, 768
    img, y, arm, ups, syn = make_inputs(arch, H, W)
    p = B.Problem(H, W, B.Arch(*arch), B.CC_QUANT_ROUND, 1e-3)
    na, nu, ns = arm.size, ups.size, syn.size
    ny = y.size
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(np.concatenate([y, arm, ups, syn])).to(dev)
    grad = torch.zeros_like(theta)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    step = torch.zeros(2, dtype=torch.int32, device=dev)
    x = torch.from_numpy(img).to(dev).reshape(-1)
    loss4 = torch.zeros(4, device=dev)
    ws = B.workspace(p, B.CC_WS_BACKWARD, device=dev)
    stream = torch.cuda.current_stream()

    def one_step():  # backward + Adam, the update fused into the gradient reductions
        B.coolchic_train_step(p, x, None, 1.0, loss4, theta, grad, m, v, step, lr=1e-2, ws=ws, stream=stream)

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    loss_start = loss4.clone()

    # Per-launch kernel timing with HIP events on the library's stream: the
    # library records a pair of its timing events (timestamps without the
    # system-scope cache fence of a default event) around the named kernel's
    # launch in every timed iteration.
    K = args.steps
    st_ev = [(B.TimingEvent(), B.TimingEvent()) for _ in range(K)]
    t_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t_ev[0].record(stream)
    t_wall = time.perf_counter()
    for k in range(K):
        # alternate the timed stage so both kernels are covered over the run
        if k % 2 == 0:
            B.coolchic_set_stage_events(B.CC_STAGE_ARM, st_ev[k][0].handle, st_ev[k][1].handle)
        else:
            B.coolchic_set_stage_events(B.CC_STAGE_SYNTHESIS, st_ev[k][0].handle, st_ev[k][1].handle)
        one_step()
    B.coolchic_set_stage_events(B.CC_STAGE_NONE)
    t_ev[1].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = t_ev[0].elapsed_time(t_ev[1])
    arm_ms = [st_ev[k][0].elapsed_ms(st_ev[k][1]) for k in range(0, K, 2)]
    syn_ms = [st_ev[k][0].elapsed_ms(st_ev[k][1]) for k in range(1, K, 2)]
    l4 = loss4.cpu().numpy()
    if l4[3] != 0.0 or not np.isfinite(l4[0]):
        print(f"non-finite loss during the timed run: {l4}", file=sys.stderr)
        sys.exit(3)

    cnt = algorithmic_counts(arch, H, W)
    ms_per_step = total_ms / K
    value = 1000.0 / ms_per_step
    arm_avg_ms = float(np.mean(arm_ms))
    syn_avg_ms = float(np.mean(syn_ms)) if syn_ms else float("nan")
    arm_tflops = cnt["arm_flop"] / (arm_avg_ms * 1e-3) / 1e12
    pass_tflops = cnt["iter_flop"] * value / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "H": H, "W": W, "latents": cnt["n_lat"],
                   "kappa_dec_mac_per_px": round(cnt["kappa_dec"], 1), "quantiser": "round+STE",
                   "step": "coolchic_backward + coolchic_adam_step"},
        "roofline": {"bound": "mfma", "kernel": "arm_kernel (ARM forward+backward, fp32 MFMA 32x32x2)",
                     "achieved": round(arm_tflops, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(arm_tflops / FP32_PEAK_TFLOPS, 4),
                     "traffic": arm_traffic_from_profile(args.workload),
                     "avg_launch_ms": round(arm_avg_ms, 5),
                     "algorithmic_flop_per_launch": cnt["arm_flop"]},
        "pass": {"iter_flop": cnt["iter_flop"], "achieved_tflops": round(pass_tflops, 2),
                 "frac_fp32_roofline": round(pass_tflops / FP32_PEAK_TFLOPS, 4),
                 "synthesis_kernel_avg_ms": round(syn_avg_ms, 5),
                 "loss_after_warmup": float(loss_start[0]), "loss_end": float(l4[0]),
                 "wall_s": round(t_wall, 3)},
    }
    if args.batch_iters > 0:
        out["batched"] = run_batched(B, args.batch_iters,
                                     log=lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_warm_start:
        out["warm_start"] = run_warm_start(warm_images, log=lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(arch, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
