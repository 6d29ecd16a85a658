"""Warm-start experiment: train the network on plain-overfit pairs, then
compare, on held-out images, how many iterations and seconds the encoder
needs to reach the plain encoder's final loss from the trained warm start,
from an untrained network of the same shape, and from scratch.

    python -m paper_2403_11651_amd.warmstart_eval --train 2000 --heldout 100 \\
        --iters 1000 --epochs 20 --out result.json

Images: the seeded blob-plus-noise generator (200 blobs per 768x512 of area);
training images use seeds 10000 + i, held-out images 20000 + i.  Every
overfit uses the low-complexity decoder, lambda 1e-3, Adam lr 1e-2, the
rounding quantiser, latents starting at 0 and decoder parameters starting
from one shared seeded draw.

Criterion for a warm-started image: it stops at the first check (every 10
iterations, rounding-mode loss) where its PSNR is within 0.1 dB of the plain
result and its rate at most 1 % above it (the first check where its loss is
at or below the plain final loss is reported too).  An image that never gets
there keeps the plain result (the fallback) and is counted with the plain
encoder's iterations plus those it spent.

The network is trained first on the pairs (regression to the plain-overfit
latents and decoder parameters), then optionally fine-tuned through the
codec's own rate-distortion loss (the non-overfitted training of Section
IV-B); both stages are evaluated.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np

from . import workloads as WL


def _image(args):
    seed, H, W = args
    return WL.image(seed, H, W, max(1, round(200 * H * W / (768 * 512))))


def make_images(seeds, H, W, workers=None):
    """Seeded images, generated in worker processes (call before the GPU is
    initialised in this process)."""
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(seeds) < 8:
        return np.stack([_image((s, H, W)) for s in seeds])
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return np.stack(list(ex.map(_image, [(s, H, W) for s in seeds], chunksize=4)))


def run(train_imgs, held_imgs, iters, epochs, rd_epochs=0, arch=None, batch=16, chunk=32, lr_net=1e-3,
        lr_rd=3e-4, log=None, check_every=10, schedules=((0, 2e-3), (30, 2e-3), (30, 5e-3), (100, 1e-2)),
        load_net=None, save_net=None):
    import torch
    from . import binding as B
    from . import warmstart as WSt
    arch = arch or B.LOW
    log = log or (lambda m: None)
    dev = torch.device("cuda")
    H, W = held_imgs.shape[-2:]
    n_ho = len(held_imgs)
    n_lat = B.latent_count(B.Problem(H, W, arch))
    n_theta = sum(B.param_count(arch))
    px = H * W
    out = {"H": int(H), "W": int(W), "heldout": n_ho, "plain_iters": iters, "epochs": epochs,
           "rd_epochs": rd_epochs, "batch": batch}
    models = {}
    if load_net is not None:
        net = WSt.WarmStart(arch, H, W, seed=1, device=dev)
        net.net.copy_(torch.from_numpy(np.load(load_net)))
        models["loaded"] = net
        out["loaded_net"] = True
    else:
        # 1. training pairs from the plain encoder
        n_tr = len(train_imgs)
        out["train_pairs"] = n_tr
        t0 = time.perf_counter()
        y_t = torch.empty(n_tr, n_lat, device=dev)
        th_t = torch.empty(n_tr, n_theta, device=dev)
        for s in range(0, n_tr, chunk):
            e = min(n_tr, s + chunk)
            ys, ths, _, _ = WSt.plain_overfit(arch, list(train_imgs[s:e]), iters)
            y_t[s:e] = torch.from_numpy(ys).to(dev)
            th_t[s:e] = torch.from_numpy(ths).to(dev)
            log(f"pairs {e}/{n_tr}: {time.perf_counter() - t0:.1f} s")
        out["pair_generation_s"] = round(time.perf_counter() - t0, 2)
        # 2. train the network on the pairs (pi starts at the mean target)
        x_tr = torch.from_numpy(np.ascontiguousarray(train_imgs)).to(dev)
        net = WSt.WarmStart(arch, H, W, seed=1, pi=th_t.mean(0).cpu().numpy(), device=dev)
        t0 = time.perf_counter()
        hist = net.train(x_tr, y_t, th_t, epochs, batch=batch, lr=lr_net, log=log)
        torch.cuda.synchronize()
        out["train_s"] = round(time.perf_counter() - t0, 2)
        out["train_loss"] = [round(h, 6) for h in hist]
        del y_t, th_t
        models["pairs_only"] = net
        if rd_epochs:
            # fine-tune copies through the codec's loss, with either proxy
            for tag, quant in (("rd_round", B.CC_QUANT_ROUND), ("rd_noise", B.CC_QUANT_NOISE)):
                m = WSt.WarmStart(arch, H, W, seed=1, device=dev)
                m.net.copy_(net.net)
                t0 = time.perf_counter()
                rd = m.train_rd(x_tr, rd_epochs, batch=batch, lr=lr_rd, quant=quant, log=log)
                torch.cuda.synchronize()
                out[f"{tag}_train_s"] = round(time.perf_counter() - t0, 2)
                out[f"{tag}_train_loss"] = [round(h, 6) for h in rd]
                models[tag] = m
        net = models.get("rd_round", net)
        del x_tr
        if save_net:
            np.save(save_net, net.net.cpu().numpy())
    models["untrained"] = WSt.WarmStart(arch, H, W, seed=1, pi=WSt.decoder_init(7, arch), device=dev)

    # 3. held-out: plain from scratch, then warm starts
    held = list(held_imgs)
    _, _, L_plain, t_plain = WSt.plain_overfit(arch, held, iters)
    it_time = t_plain / iters  # seconds per iteration of the whole held-out batch
    p_psnr, p_bpp = WSt.psnr(L_plain[:, 1]), L_plain[:, 2] / px
    res = {"plain": {"iters": iters, "s_per_image": t_plain / n_ho, "loss_mean": float(L_plain[:, 0].mean()),
                     "psnr_mean": float(p_psnr.mean()), "bpp_mean": float(p_bpp.mean())}}
    x_ho = torch.from_numpy(np.ascontiguousarray(held_imgs)).to(dev)
    na, nu, _ = B.param_count(arch)
    per_img_iter = it_time / n_ho
    for mname, model in models.items():
        for nz, lr in (schedules if mname != "untrained" else schedules[-1:]):
            name = f"{mname}_noise{nz}_lr{lr:g}"
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            y0, th0 = model.predict(x_ho, batch=batch)
            torch.cuda.synchronize()
            t_pred = time.perf_counter() - t0
            y0, th0 = y0.cpu().numpy(), th0.cpu().numpy()
            enc = WSt.encoder(arch, held, list(y0), [(t[:na], t[na:na + nu], t[na + nu:]) for t in th0], lr=lr)
            enc.probe()
            torch.cuda.synchronize()
            L0 = enc.loss.cpu().numpy()
            r = WSt.iterations_to_target(enc, L_plain[:, 0], p_psnr, p_bpp, px, iters, check_every, noise_iters=nz)
            hl, hc = r["loss"], r["criterion"]
            ok = hc >= 0
            # seconds per image: its share of the prediction, plus its own
            # iterations at the batch's per-image iteration cost; an image that
            # never meets the criterion falls back to the plain encoder
            secs = t_pred / n_ho + np.where(ok, hc, iters) * per_img_iter + np.where(ok, 0.0, t_plain / n_ho)
            res[name] = {"criterion_met": int(ok.sum()), "fallbacks": int((~ok).sum()),
                         "iters_median_criterion": float(np.median(hc[ok])) if ok.any() else None,
                         "iters_mean_criterion": float(hc[ok].mean()) if ok.any() else None,
                         "met_at_start": int((hc == 0).sum()),
                         "loss_reached": int((hl >= 0).sum()),
                         "iters_median_loss": float(np.median(hl[hl >= 0])) if (hl >= 0).any() else None,
                         "start_loss_mean": float(L0[:, 0].mean()), "start_psnr_mean": float(WSt.psnr(L0[:, 1]).mean()),
                         "predict_s_per_image": t_pred / n_ho, "s_per_image": float(secs.mean()),
                         "run_s": round(r["seconds"], 3), "noise_iters": nz, "lr": lr}
            log(f"{name}: {res[name]}")
            del enc
    out["heldout_results"] = res
    best = min((k for k in res if not k.startswith(("plain", "untrained"))), key=lambda k: res[k]["s_per_image"])
    out["best_warm_variant"] = best
    out["s_per_image_plain"] = res["plain"]["s_per_image"]
    out["s_per_image_warm"] = res[best]["s_per_image"]
    out["speedup_warm_vs_plain"] = res["plain"]["s_per_image"] / res[best]["s_per_image"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--heldout", type=int, default=100)
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--rd-epochs", type=int, default=20)
    ap.add_argument("--save-net", default="")
    ap.add_argument("--load-net", default="")
    ap.add_argument("--H", type=int, default=512)
    ap.add_argument("--W", type=int, default=768)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    n_tr = 0 if args.load_net else args.train
    tr = make_images([10000 + i for i in range(n_tr)], args.H, args.W) if n_tr else None
    ho = make_images([20000 + i for i in range(args.heldout)], args.H, args.W)
    t_gen = time.perf_counter() - t0
    log(f"images generated in {t_gen:.1f} s")
    res = run(tr, ho, args.iters, args.epochs, rd_epochs=args.rd_epochs, log=log,
              load_net=args.load_net or None, save_net=args.save_net or None)
    res["image_generation_s"] = round(t_gen, 2)
    txt = json.dumps(res)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
