"""Learned warm start for the overfitting encoder.

Section IV-B trains an analysis transform that maps an image to the latent
grids (and learns the decoder parameters beside it); Section V suggests
fine-tuning such an output per image instead of overfitting from scratch.
Here a small network (four bfloat16 stride-2 convolutions and per-level
heads, see include/coolchic.h) predicts both the latent pyramid and the
decoder parameters of an image; it is trained on pairs (image, result of the
plain from-scratch overfitting of that image), and the encoder then starts
from its prediction.  The plain overfit stays the fallback: an image whose
warm-started run does not reach the plain result keeps the plain result.

Everything on the GPU runs in the library's kernels: the network's forward
and backward (coolchic_warm_forward / coolchic_warm_backward), Adam, and the
overfitting itself (the batched encoder).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as B
from . import workloads as WL
from .batch import BatchEncoder

N_CH = 32


def init_blocks(n_theta):
    """(count, std) of each block of the packed master parameters, in layout
    order: He-normal conv kernels, small head weights, zero biases."""
    blocks = []
    for k in range(1, 5):
        cin = 3 if k == 1 else N_CH
        blocks += [(N_CH * 9 * cin, float(np.sqrt(2.0 / (9 * cin)))), (N_CH, 0.0)]
    hv = 0.1 / np.sqrt(N_CH)
    blocks += [(N_CH, hv), (1, 0.0), (27, 0.1 / np.sqrt(27))]
    for _ in range(1, 7):
        blocks += [(N_CH, hv), (1, 0.0)]
    blocks += [(n_theta * N_CH, hv), (n_theta, 0.0)]
    return blocks


def decoder_init(seed, arch):
    """Initial decoder parameters of a from-scratch overfit (all images share
    them): N(0, 0.1^2)."""
    return WL.weights(seed, sum(B.param_count(arch)))


class WarmStart:
    """The warm-start network for images of one size (H, W multiples of 64)."""

    def __init__(self, arch=B.LOW, H=512, W=768, seed=0, pi=None, device="cuda"):
        self.arch, self.H, self.W = arch, H, W
        self.device = torch.device(device)
        self.n_theta = sum(B.param_count(arch))
        self.n_lat = B.latent_count(B.Problem(H, W, arch))
        net = WL.normal_blocks(seed, init_blocks(self.n_theta))
        if pi is not None:
            net[-self.n_theta:] = pi
        if net.size != B.warm_param_count(arch):
            raise RuntimeError("warm-start parameter layout mismatch")
        self.net = torch.from_numpy(net).to(self.device)
        self.m = torch.zeros_like(self.net)
        self.v = torch.zeros_like(self.net)
        self.g = torch.zeros_like(self.net)
        self.step_ctr = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.loss4 = torch.zeros(4, device=self.device)
        self._ws = {}

    def _wsp(self, batch, which):
        key = (batch, which)
        if key not in self._ws:
            self._ws[key] = B.warm_workspace(B.WarmProblem(self.H, self.W, batch, self.arch), which, self.device)
        return self._ws[key]

    def predict(self, x, batch=16):
        """x [N][3][H][W] (device) -> (y [N][n_lat], theta [N][n_theta])."""
        n = x.shape[0]
        y = torch.empty(n, self.n_lat, device=self.device)
        th = torch.empty(n, self.n_theta, device=self.device)
        for s in range(0, n, batch):
            e = min(n, s + batch)
            wp = B.WarmProblem(self.H, self.W, e - s, self.arch)
            B.coolchic_warm_forward(wp, x[s:e], self.net, y[s:e], th[s:e], ws=self._wsp(e - s, B.CC_WS_FORWARD))
        return y, th

    def loss_and_grad(self, x, y_t, th_t):
        """Batch loss (device loss4) and gradient (self.g) of x [b][3][H][W]."""
        b = x.shape[0]
        wp = B.WarmProblem(self.H, self.W, b, self.arch)
        B.coolchic_warm_backward(wp, x, self.net, y_t, th_t, self.loss4, self.g, ws=self._wsp(b, B.CC_WS_BACKWARD))
        return self.loss4

    def train(self, x, y_t, th_t, epochs, batch=16, lr=1e-3, log=None):
        """Adam on the training pairs, mini-batches taken in order (the pairs
        are independent draws); returns the mean loss of every epoch."""
        n = (x.shape[0] // batch) * batch
        if n == 0:
            raise ValueError("fewer training pairs than one mini-batch")
        hist = []
        for ep in range(epochs):
            acc = torch.zeros((), device=self.device)
            for s in range(0, n, batch):
                self.loss_and_grad(x[s:s + batch], y_t[s:s + batch], th_t[s:s + batch])
                acc += self.loss4[0]
                B.coolchic_adam_step(self.net, self.g, self.m, self.v, self.step_ctr, lr=lr)
            hist.append(float(acc) / (n // batch))
            if log:
                log(f"warm-start epoch {ep}: loss {hist[-1]:.5f}")
        return hist


    def train_rd(self, x, epochs, batch=16, lr=3e-4, lam=1e-3, quant=B.CC_QUANT_ROUND, noise_seed=11, log=None):
        """Fine-tunes the network through the codec: the loss of a mini-batch is
        the mean over its images of Eq. (1) evaluated at the predicted latents
        and decoder (rounding with the straight-through gradient, or the noise
        proxy with fresh noise every step), its output gradients come from the
        batched coolchic backward pass, and coolchic_warm_backward_grad carries
        them into the network (the non-overfitted training of Section IV-B,
        started from the pair regression).  Returns the mean loss of every
        epoch."""
        n = (x.shape[0] // batch) * batch
        if n == 0:
            raise ValueError("fewer images than one mini-batch")
        H, W, dev = self.H, self.W, self.device
        na, nu, ns = B.param_count(self.arch)
        xb = torch.empty(batch, 3, H, W, device=dev)
        yp = torch.empty(batch, self.n_lat, device=dev)
        thp = torch.empty(batch, self.n_theta, device=dev)
        gy = torch.empty(batch, self.n_lat, device=dev)
        gth = torch.empty(batch, self.n_theta, device=dev)
        u = torch.empty(batch * self.n_lat, device=dev)
        loss = torch.zeros(batch, 4, device=dev)
        noise = quant == B.CC_QUANT_NOISE
        probs = [B.Problem(H, W, self.arch, quant, lam)] * batch
        io = [dict(img=xb[k].reshape(-1), y=yp[k], u=u[k * self.n_lat:(k + 1) * self.n_lat] if noise else None,
                   arm_w=thp[k, :na],
                   ups_w=thp[k, na:na + nu], syn_w=thp[k, na + nu:], loss4=loss[k], g_y=gy[k], g_arm=gth[k, :na],
                   g_ups=gth[k, na:na + nu], g_syn=gth[k, na + nu:]) for k in range(batch)]
        plan = B.BatchPlan(probs, io, dloss=1.0 / batch, device=dev)
        wp = B.WarmProblem(H, W, batch, self.arch)
        hist = []
        for ep in range(epochs):
            acc = torch.zeros((), device=dev)
            for s in range(0, n, batch):
                xb.copy_(x[s:s + batch])
                B.coolchic_warm_forward(wp, xb, self.net, yp, thp, ws=self._wsp(batch, B.CC_WS_FORWARD))
                if noise:
                    B.coolchic_uniform_noise(u, noise_seed, step=self.step_ctr)
                plan.backward()
                B.coolchic_warm_backward_grad(wp, xb, self.net, gy, gth, self.loss4, self.g,
                                              ws=self._wsp(batch, B.CC_WS_BACKWARD))
                B.coolchic_adam_step(self.net, self.g, self.m, self.v, self.step_ctr, lr=lr)
                acc += loss[:, 0].sum() / batch
            hist.append(float(acc) / (n // batch))
            if log:
                log(f"warm-start rate-distortion epoch {ep}: loss {hist[-1]:.5f}")
        plan.close()
        return hist


# ---- encoding with and without the warm start -----------------------------

def encoder(arch, images, y0, params0, lam=1e-3, lr=1e-2):
    """A batched encoder (rounding quantiser) over same-size images."""
    H, W = images[0].shape[-2:]
    probs = [B.Problem(H, W, arch, B.CC_QUANT_ROUND, lam) for _ in images]
    return BatchEncoder(probs, images, y0, params0, lr=lr)


def plain_overfit(arch, images, iters, dec_seed=7, graph_steps=50, lam=1e-3, noise_frac=0.8):
    """From-scratch overfitting: latents 0, decoder parameters from the shared
    seeded initialisation, the noise proxy for the first noise_frac of the
    iterations and rounding for the rest.  Returns (y [n][n_lat], theta
    [n][n_theta], loss4 [n][4] of the final parameters with rounding,
    seconds)."""
    H, W = images[0].shape[-2:]
    n_lat = B.latent_count(B.Problem(H, W, arch))
    na, nu, ns = B.param_count(arch)
    w = decoder_init(dec_seed, arch)
    params0 = [(w[:na], w[na:na + nu], w[na + nu:])] * len(images)
    enc = encoder(arch, images, [np.zeros(n_lat, np.float32)] * len(images), params0, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    enc.fit(iters, noise_frac=noise_frac, graph_steps=graph_steps)
    enc.backward()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ys = np.stack([enc.params(k)[0] for k in range(len(images))])
    ths = np.stack([np.concatenate(enc.params(k)[1:]) for k in range(len(images))])
    return ys, ths, enc.loss.cpu().numpy(), secs


def psnr(mse):
    return -10.0 * np.log10(np.maximum(mse, 1e-30))


def iterations_to_target(enc, target_loss, target_psnr, target_bpp, px, max_iters, check_every=10, noise_iters=0):
    """Runs enc (the noise proxy for the first noise_iters iterations, then
    rounding), checking every check_every iterations the rounding-mode loss4
    of each image (the first check is the starting point itself), until
    every image meets the criterion: PSNR within 0.1 dB of target_psnr[k]
    and rate at most 1 % above target_bpp[k] (px pixels per image).
    Returns dict(loss=iterations at which the loss first is at or below
    target_loss[k], criterion=iterations at which the criterion first holds
    (-1: never), at=loss4 rows there, seconds)."""
    n = len(target_loss)
    hit_l = np.full(n, -1)
    hit_c = np.full(n, -1)
    at = np.zeros((n, 4), np.float32)
    graphs = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0

    def check():
        L = enc.loss.cpu().numpy()
        hit_l[(hit_l < 0) & (L[:, 0] <= target_loss)] = done
        ok = (psnr(L[:, 1]) >= target_psnr - 0.1) & (L[:, 2] / px <= 1.01 * target_bpp)
        new = (hit_c < 0) & ok
        hit_c[new] = done
        at[new] = L[new]

    enc.probe()  # the prediction itself (iteration 0)
    check()
    while done < max_iters and (hit_c < 0).any():
        mode = B.CC_QUANT_NOISE if done < noise_iters else B.CC_QUANT_ROUND
        if mode not in graphs:
            enc.set_mode(mode)
            graphs[mode] = enc.capture(check_every, probe=True)
        enc.set_mode(mode)
        graphs[mode].replay()
        done += check_every
        check()
    torch.cuda.synchronize()
    return dict(loss=hit_l, criterion=hit_c, at=at, seconds=time.perf_counter() - t0)
