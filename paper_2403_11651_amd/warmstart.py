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


# ---- encoding with and without the warm start -----------------------------

def encoder(arch, images, y0, params0, lam=1e-3, lr=1e-2):
    """A batched encoder (rounding quantiser) over same-size images."""
    H, W = images[0].shape[-2:]
    probs = [B.Problem(H, W, arch, B.CC_QUANT_ROUND, lam) for _ in images]
    return BatchEncoder(probs, images, y0, params0, lr=lr)


def plain_overfit(arch, images, iters, dec_seed=7, graph_steps=50, lam=1e-3):
    """From-scratch overfitting: latents 0, decoder parameters from the shared
    seeded initialisation.  Returns (y [n][n_lat], theta [n][n_theta], loss4
    [n][4] of the final parameters, seconds)."""
    H, W = images[0].shape[-2:]
    n_lat = B.latent_count(B.Problem(H, W, arch))
    na, nu, ns = B.param_count(arch)
    w = decoder_init(dec_seed, arch)
    params0 = [(w[:na], w[na:na + nu], w[na + nu:])] * len(images)
    enc = encoder(arch, images, [np.zeros(n_lat, np.float32)] * len(images), params0, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    enc.run(iters, graph_steps=graph_steps)
    enc.backward()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ys = np.stack([enc.params(k)[0] for k in range(len(images))])
    ths = np.stack([np.concatenate(enc.params(k)[1:]) for k in range(len(images))])
    return ys, ths, enc.loss.cpu().numpy(), secs


def iterations_to_target(enc, target, max_iters, check_every=10):
    """Runs enc until each image's loss is at or below target[k] (checked
    every check_every iterations, on the loss of the parameters the last
    iteration of the block started from).  Returns (iterations per image,
    -1 where never reached; the loss4 rows at the crossing; seconds)."""
    n = len(target)
    hit = np.full(n, -1)
    at = np.zeros((n, 4), np.float32)
    g = enc.capture(check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < max_iters and (hit < 0).any():
        g.replay()
        done += check_every
        L = enc.loss.cpu().numpy()
        new = (hit < 0) & (L[:, 0] <= target)
        hit[new] = done
        at[new] = L[new]
    torch.cuda.synchronize()
    return hit, at, time.perf_counter() - t0
