"""Plain float64 NumPy definition of the non-overfitted analysis transform.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section IV-B ("Non-overfitted Cool-chic", Fig. 6, Eq. (3)): an analysis
transform maps the image straight to the L = 7 latent grids of Cool-chic,
y_hat = Q(f_alpha(x)), so that encoding is one forward pass.  The paper gives
its structure in words (the figure itself is not available):

* a series of ConvNeXt-style residual blocks with C = 64 features
  progressively downsamples the image; the first block does not downsample;
* a downsampling block complements its identity branch with a stride-2 2x2
  average pooling and a 1x1 convolution;
* further residual blocks follow each downsampling;
* after each downsampling step a 1x1 convolution turns the C features into
  the latent grid of that resolution.

Reading used here (the choices the text leaves open):

* ConvNeXt block (c_in -> C, stride s): depth-wise 7x7 convolution of the
  input (zero padding 3, stride s, with bias), layer normalisation over the
  c_in channels of each position (eps 1e-6, per-channel scale and shift),
  a 1x1 convolution c_in -> 4C with bias, GELU (the erf form), a 1x1
  convolution 4C -> C with bias; the block output adds the identity branch:
  the input itself when c_in = C and s = 1, otherwise a 1x1 convolution
  c_in -> C (with bias) of the input, average-pooled 2x2 with stride 2 when
  s = 2;
* level 0: block 3 -> 64 (stride 1), then E = 2 blocks 64 -> 64; levels
  l = 1..6: block 64 -> 64 (stride 2), then E = 2 blocks; 21 blocks in all;
* latent l = 1x1 convolution 64 -> 1 (with bias) of the level's last block
  output, at resolution (H / 2^l, W / 2^l) (H, W multiples of 64).

That is 126.6 kMAC per image pixel (mac_per_pixel), against the 130 000 the
paper's complexity plot shows for N-O Cool-chic (its text says 160 k).

Precision model (the rounding points of the gfx950 kernels, whose 1x1
convolutions run on the bfloat16 matrix cores with float32 accumulation):
the 1x1 convolution weights are used rounded to bfloat16; so are their
inputs -- the layer-normalised features, the GELU output, the image (for the
first block's identity branch) and the pooled input of a downsampling
identity branch; every block output is stored rounded to bfloat16.  The
depth-wise convolution, the normalisation, GELU, biases and the latent heads
are float32 on the GPU, float64 here.  ``round_bf16=False`` removes every
rounding.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

from .warmstart import bf16

C = 64            # features
EXP = 4           # hidden expansion of the block's 1x1 convolutions
K = 7             # depth-wise kernel side
E = 2             # blocks after each level's first block
L = 7             # latent grids
LN_EPS = 1e-6


def block_specs():
    """(level, c_in, stride, is_last_of_level) of the 21 blocks, in order."""
    out = []
    for l in range(L):
        out.append((l, 3 if l == 0 else C, 1 if l == 0 else 2, False))
        for e in range(E):
            out.append((l, C, 1, e == E - 1))
    return out


def block_param_sizes(c_in, stride):
    """Sizes of (dw_w, dw_b, ln_g, ln_b, W1, b1, W2, b2, Wid, bid) of a block
    (Wid, bid empty for a plain identity)."""
    ident = c_in != C or stride != 1
    return [c_in * K * K, c_in, c_in, c_in, EXP * C * c_in, EXP * C, C * EXP * C, C,
            C * c_in if ident else 0, C if ident else 0]


def param_count():
    """Parameters of the whole transform: the blocks in order, then per level
    the head (64 weights and a bias)."""
    n = sum(sum(block_param_sizes(ci, s)) for _, ci, s, _ in block_specs())
    return n + L * (C + 1)


def unpack(theta):
    """Splits the flat parameter vector into per-block dicts and per-level
    heads (views into theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    names = ("dw_w", "dw_b", "ln_g", "ln_b", "W1", "b1", "W2", "b2", "Wid", "bid")
    blocks, o = [], 0
    for l, ci, s, last in block_specs():
        d = {"level": l, "c_in": ci, "stride": s, "last": last}
        for nm, n in zip(names, block_param_sizes(ci, s)):
            d[nm] = theta[o:o + n]
            o += n
        d["dw_w"] = d["dw_w"].reshape(ci, K, K)
        d["W1"] = d["W1"].reshape(EXP * C, ci)
        d["W2"] = d["W2"].reshape(C, EXP * C)
        if d["Wid"].size:
            d["Wid"] = d["Wid"].reshape(C, ci)
        blocks.append(d)
    heads = []
    for l in range(L):
        heads.append((theta[o:o + C], theta[o + C]))
        o += C + 1
    assert o == theta.size
    return blocks, heads


def mac_per_pixel(H=512, W=768):
    """Multiply-accumulates per image pixel of one forward pass."""
    total = 0
    for l, ci, s, _ in block_specs():
        n_out = (H >> l) * (W >> l)
        ident = ci * C if (ci != C or s != 1) else 0
        total += n_out * (ci * K * K + EXP * C * ci + C * EXP * C + ident)
    for l in range(L):
        total += (H >> l) * (W >> l) * C
    return total / (H * W)


# ------------------------------------------------------------------ layers

def dwconv(x, w, b, stride):
    """Depth-wise K x K convolution (cross-correlation), zero padding K // 2:
    out[c][i][j] = b[c] + sum_{dy, dx} w[c][dy][dx] x[c][s i + dy - 3][s j + dx - 3]."""
    c, h, wd = x.shape
    p = K // 2
    xp = np.zeros((c, h + 2 * p, wd + 2 * p))
    xp[:, p:p + h, p:p + wd] = x
    ho, wo = (h + stride - 1) // stride, (wd + stride - 1) // stride
    out = np.zeros((c, ho, wo))
    for dy in range(K):
        for dx in range(K):
            patch = xp[:, dy:dy + stride * (ho - 1) + 1:stride, dx:dx + stride * (wo - 1) + 1:stride]
            out += w[:, dy, dx][:, None, None] * patch
    return out + b[:, None, None]


def layer_norm(x, g, b):
    """Normalisation over the channels of each position: (x - mean) /
    sqrt(var + eps) * g + b, var the biased variance."""
    mu = x.mean(axis=0, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=0, keepdims=True)
    return (x - mu) / np.sqrt(var + LN_EPS) * g[:, None, None] + b[:, None, None]


def gelu(x):
    """x Phi(x) with Phi the standard normal CDF (the erf form)."""
    return 0.5 * x * (1.0 + scipy.special.erf(x / math.sqrt(2.0)))


def conv1x1(W, x, b=None):
    """out[o] = sum_i W[o][i] x[i] (+ b[o]) at every position."""
    out = np.einsum("oi,ihw->ohw", W, x)
    return out if b is None else out + b[:, None, None]


def avgpool2(x):
    """2x2 average pooling with stride 2."""
    c, h, w = x.shape
    return x.reshape(c, h // 2, 2, w // 2, 2).mean(axis=(2, 4))


def block(x, p, round_bf16=True):
    """One ConvNeXt-style residual block (see the module docstring)."""
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    t = layer_norm(dwconv(x, p["dw_w"], p["dw_b"], p["stride"]), p["ln_g"], p["ln_b"])
    h = gelu(conv1x1(R(p["W1"]), R(t), p["b1"]))
    m = conv1x1(R(p["W2"]), R(h), p["b2"])
    if p["Wid"].size:
        src = avgpool2(x) if p["stride"] == 2 else x
        ident = conv1x1(R(p["Wid"]), R(src), p["bid"])
    else:
        ident = x
    return R(m + ident)


def forward(x, theta, round_bf16=True):
    """x: [3][H][W] (H, W multiples of 64).  Returns (latents: list of the 7
    grids [H >> l][W >> l], features: the output of every block)."""
    x = np.asarray(x, dtype=np.float64)
    assert x.shape[0] == 3 and x.shape[1] % 64 == 0 and x.shape[2] % 64 == 0
    blocks, heads = unpack(theta)
    ys, feats = [], []
    f = x
    for p in blocks:
        f = block(f, p, round_bf16)
        feats.append(f)
        if p["last"]:
            hw, hb = heads[p["level"]]
            ys.append(np.einsum("i,ihw->hw", hw, f) + hb)
    return ys, feats


def window_latents(x, theta, level, i0, j0, n, round_bf16=True):
    """Latents [i0:i0+n][j0:j0+n] of grid `level` (< 4) computed from a window
    of the image only.  A block's output at a position depends on its input
    within 3 positions (the 7x7 depth-wise kernel; the pooled identity reads
    2q and 2q + 1), so the last block of level l depends on the image within
    9 (l = 0), 25, 57, 121 pixels of its footprint; a margin of 16 * 2^l
    pixels, aligned to 2^l so that every stride keeps its phase, covers it,
    and where the window meets the image border the zero padding is the
    image's own."""
    x = np.asarray(x, dtype=np.float64)
    s = 1 << level
    H, W = x.shape[1:]
    m = 16 * s
    r0, r1 = max(0, i0 * s - m), min(H, (i0 + n) * s + m)
    c0, c1 = max(0, j0 * s - m), min(W, (j0 + n) * s + m)
    blocks, heads = unpack(theta)
    f = x[:, r0:r1, c0:c1]
    for p in blocks:
        if p["level"] > level:
            break
        f = block(f, p, round_bf16)
    hw, hb = heads[level]
    y = np.einsum("i,ihw->hw", hw, f) + hb
    a, b = i0 - r0 // s, j0 - c0 // s
    return y[a:a + n, b:b + n]


def encode(x, theta, round_bf16=True):
    """N-O encoding (Section IV-B): the packed latent vector of Cool-chic's
    layout (level 0 first, each grid in raster order), quantised by
    rounding, and the unquantised one."""
    ys, _ = forward(x, theta, round_bf16)
    y = np.concatenate([g.ravel() for g in ys])
    return np.rint(y), y
