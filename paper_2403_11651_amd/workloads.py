"""Seeded synthetic inputs for the Cool-chic rate-distortion pass.

This module only draws random numbers in a fixed order; it holds none of the
method's arithmetic (no quantisation, context, rate, upsampling or synthesis),
so both the HIP path and the FP64 oracle can take their inputs from it.

Workloads (all FP32, NumPy PCG64 ``default_rng``):

* image: a sum of Gaussian blobs plus white noise, clipped to [0, 1].  For each
  blob the draws are, in order, the centre row, the centre column, the width
  sigma ~ U[4, 16] pixels and one amplitude per colour channel ~ U[0, 1].
  The paper's own test images (Kodak, CLIC) are not available, so these stand
  in for a natural 768x512 photograph: smooth structure at several scales and
  a noise floor the codec cannot compress.
* latents: one grid per level l of size (H/2^l, W/2^l), drawn iid from a
  Laplace(0, b_l) distribution with b_l ~ U[0.5, 3] per level.
* weights: every parameter (ARM, upsampling and synthesis, biases included)
  drawn iid from N(0, 0.1^2).
* noise: the additive quantisation noise u ~ U[-0.5, 0.5).
* normal_blocks: initial parameters of a network, block by block N(0, std^2)
  (the caller gives each block's size and std).
* analysis_params: parameters of the analysis transform, fan-in-scaled
  normal weights, small biases, layer-norm scales near 1.
"""
from __future__ import annotations

import numpy as np


def image(seed: int, H: int, W: int, n_blobs: int, noise_std: float = 0.02) -> np.ndarray:
    """Blob-plus-noise RGB image, planar [3][H][W] float32 in [0, 1]."""
    rng = np.random.default_rng(seed)
    ii = np.arange(H, dtype=np.float64)[:, None]
    jj = np.arange(W, dtype=np.float64)[None, :]
    x = np.zeros((3, H, W), dtype=np.float64)
    for _ in range(n_blobs):
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        sigma = rng.uniform(4.0, 16.0)
        amp = rng.uniform(0.0, 1.0, size=3)
        # evaluate the blob only inside a +-6 sigma window: beyond it the
        # Gaussian is below 2e-8, under FP32 resolution of the image
        r = int(np.ceil(6.0 * sigma))
        i0, i1 = max(0, int(cy) - r), min(H, int(cy) + r + 1)
        j0, j1 = max(0, int(cx) - r), min(W, int(cx) + r + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        g = np.exp(-((ii[i0:i1] - cy) ** 2 + (jj[:, j0:j1] - cx) ** 2) / (2.0 * sigma * sigma))
        x[:, i0:i1, j0:j1] += amp[:, None, None] * g[None]
    x += rng.normal(0.0, noise_std, size=x.shape)
    return np.clip(x, 0.0, 1.0).astype(np.float32)


def level_shapes(H: int, W: int, L: int):
    return [(H >> l, W >> l) for l in range(L)]


def latents(seed: int, H: int, W: int, L: int, rounded: bool = False) -> np.ndarray:
    """Packed latent pyramid (level-major, row-major), float32 [sum_l H_l W_l]."""
    rng = np.random.default_rng(seed)
    parts = []
    for (h, w) in level_shapes(H, W, L):
        b = rng.uniform(0.5, 3.0)
        parts.append(rng.laplace(0.0, b, size=(h, w)).ravel())
    y = np.concatenate(parts)
    if rounded:
        y = np.rint(y)
    return y.astype(np.float32)


def weights(seed: int, n: int, std: float = 0.1) -> np.ndarray:
    """n iid N(0, std^2) parameters, float32."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=n).astype(np.float32)


def normal_blocks(seed: int, blocks) -> np.ndarray:
    """Concatenated iid normal draws, block by block: blocks is a list of
    (count, std); a block with std 0 is zeros (and draws nothing)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n, std in blocks:
        parts.append(rng.normal(0.0, std, size=n) if std > 0 else np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def analysis_params(seed: int, c: int = 64, hid: int = 256, k: int = 7, levels: int = 7, extra: int = 2) -> np.ndarray:
    """Seeded parameters of the analysis transform in its packed layout: per
    block (the first of each level takes the image's 3 channels at level 0,
    else c, and has a 1x1 identity branch) dw_w [c_in][k][k], dw_b, ln_g,
    ln_b [c_in], W1 [hid][c_in], b1 [hid], W2 [c][hid], b2 [c], (Wid [c][c_in],
    bid [c]); then per level a head of c weights and a bias.  Weights
    N(0, 1 / fan_in), biases and shifts N(0, 0.02^2), layer-norm scales
    1 + N(0, 0.1^2), float32."""
    rng = np.random.default_rng(seed)
    parts = []
    g = lambda n, std, mean=0.0: parts.append(rng.normal(mean, std, size=n))  # noqa: E731
    for lvl in range(levels):
        for e in range(1 + extra):
            ci = 3 if (lvl == 0 and e == 0) else c
            g(ci * k * k, 1.0 / k)
            g(ci, 0.02)
            g(ci, 0.1, 1.0)
            g(ci, 0.02)
            g(hid * ci, 1.0 / np.sqrt(ci))
            g(hid, 0.02)
            g(c * hid, 1.0 / np.sqrt(hid))
            g(c, 0.02)
            if e == 0:
                g(c * ci, 1.0 / np.sqrt(ci))
                g(c, 0.02)
    for lvl in range(levels):
        g(c, 1.0 / np.sqrt(c))
        g(1, 0.02)
    return np.concatenate(parts).astype(np.float32)


def noise(seed: int, n: int) -> np.ndarray:
    """Additive quantisation noise u ~ U[-0.5, 0.5), float32."""
    rng = np.random.default_rng(seed)
    return (rng.random(n) - 0.5).astype(np.float32)


def batch_sizes(seed: int, n: int):
    """n image sizes (H, W): W ~ U{256, 320, ..., 1024}, H ~ U{256, ..., 768}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        w = 64 * int(rng.integers(4, 17))
        h = 64 * int(rng.integers(4, 13))
        out.append((h, w))
    return out


# The fixed seeds of the named workloads.
SEEDS = {
    "tiny": dict(image=0, latents=1, weights=2, noise=4),
    "fd16": dict(image=3, latents=3, weights=3, noise=3),
    "full": dict(image=10, latents=11, weights=12, noise=13),
    "low": dict(image=10, latents=11, weights=12, noise=13),
}
