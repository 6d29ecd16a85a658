"""Seeded parity cases shared by the GPU tests (inputs only, no arithmetic)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from paper_2403_11651_amd import workloads as WL


@dataclass
class Case:
    name: str
    H: int
    W: int
    arch: tuple          # (n_levels, arm_ctx, arm_layers, ups_taps, syn_hidden, syn_res)
    img: np.ndarray
    y: np.ndarray
    u: np.ndarray | None
    arm: np.ndarray
    ups: np.ndarray
    syn: np.ndarray
    lam: float = 1e-3


def sizes(arch):
    """(n_arm, n_ups, n_syn) of an architecture tuple (n_levels, arm_ctx,
    arm_layers, ups_taps, syn_hidden, syn_res[, ups_shared])."""
    L, C, NH, K, Hs, R = arch[:6]
    shared = len(arch) > 6 and arch[6]
    n_ups = 0 if L < 2 else (K * K if shared else (L - 1) * 2 * K)
    return NH * (C * C + C) + 2 * C + 2, n_ups, Hs * L + Hs + 3 * Hs + 3 + R * 84


def n_latents(H, W, L):
    return sum((H >> l) * (W >> l) for l in range(L))


def make(name, H, W, arch, seeds=(0, 1, 2, 4), n_blobs=12, rounded=False, noise=False, lam=1e-3, wstd=0.1):
    si, sl, sw, su = seeds
    L = arch[0]
    na, nu, ns = sizes(arch)
    w = WL.weights(sw, na + nu + ns, std=wstd)
    n_lat = n_latents(H, W, L)
    return Case(name, H, W, arch, WL.image(si, H, W, n_blobs), WL.latents(sl, H, W, L, rounded=rounded),
                WL.noise(su, n_lat) if noise else None, w[:na], w[na:na + nu], w[na + nu:], lam)


TINY = (7, 8, 2, 8, 16, 1)
LOW = (7, 8, 2, 8, 16, 1)
FULL = (7, 24, 2, 8, 40, 2)


def tiny():
    """64x64, 12 blobs, rounded 7-level latents, 8-neighbour ARM 8-8-8-2,
    synthesis 7-16-3 + one residual conv."""
    return make("tiny64", 64, 64, TINY, seeds=(0, 1, 2, 4), n_blobs=12, rounded=True)


def low():
    """768x512 (H=512, W=768), 200 blobs, Laplace latents, low-complexity decoder."""
    return make("low768x512", 512, 768, LOW, seeds=(10, 11, 12, 13), n_blobs=200)


def full():
    """768x512, 200 blobs, Laplace latents, 24-neighbour ARM and 7-40-3 + 2 residual convs."""
    return make("full768x512", 512, 768, FULL, seeds=(10, 11, 12, 13), n_blobs=200)


def small_variants():
    """Small cases spanning several tiles, ragged tiles and every compiled
    architecture axis."""
    out = [
        make("fd16_L5", 16, 16, (5, 8, 2, 8, 16, 1), seeds=(3, 3, 3, 3), n_blobs=4, noise=True),
        make("ragged_L7_64x192", 64, 192, (7, 24, 2, 8, 40, 2), seeds=(20, 21, 22, 23)),
        make("ragged_L6_96x160_noise", 96, 160, (6, 16, 1, 8, 24, 2), seeds=(24, 25, 26, 27), noise=True),
        make("L2_8x24", 8, 24, (2, 8, 3, 8, 8, 1), seeds=(28, 29, 30, 31), n_blobs=3),
        make("L7_128x64_c24h3", 128, 64, (7, 24, 3, 8, 48, 1), seeds=(32, 33, 34, 35)),
        make("L4_40x72_c16", 40, 72, (4, 16, 2, 8, 32, 2), seeds=(36, 37, 38, 39), n_blobs=5),
        # a single latent grid: no upsampling, the synthesis sees y_hat_0 alone
        make("L1_16x40", 16, 40, (1, 8, 2, 8, 16, 1), seeds=(40, 41, 42, 43), n_blobs=3),
        make("L1_72x136_c24_noise", 72, 136, (1, 24, 2, 8, 40, 2), seeds=(44, 45, 46, 47), n_blobs=6, noise=True),
    ]
    return out
