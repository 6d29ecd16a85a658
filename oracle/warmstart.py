"""Plain float64 NumPy definition of the learned warm-start network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section IV-B ("Non-overfitted Cool-chic") replaces overfitting by an analysis
transform that maps the image to the hierarchical latent grids, one 1x1
convolution per grid on features of matching resolution, with the decoder
parameters learned beside it; Section V proposes to fine-tune such an
analysis output and decoder per image instead of overfitting from scratch.
The warm start follows that suggestion with a small network:

* trunk: four 3x3 convolutions with stride 2, zero padding 1, 32 output
  channels and ReLU: x (3 x H x W) -> f_1 (H/2) -> f_2 -> f_3 -> f_4 (H/16);
* latent heads: y_l = V_l . f_l + beta_l (1x1, 32 -> 1) for l = 1..4;
  y_5 and y_6 from f_4 average-pooled by 2 and by 4; y_0 = a 3x3 convolution
  of x (zero padding) + beta_0 + V_0 . f_1 repeated over each 2x2 block;
* decoder-parameter head: theta = P . mean(f_4) + pi (global average pool,
  then a linear map to the n_theta parameters the decoder architecture has).

Precision model (the same rounding points as the gfx950 kernels): the
matrix-core operands are bfloat16 -- the image and every feature map f_k are
rounded to bfloat16 (round to nearest, ties to even), every weight matrix
(conv kernels, V, P, the level-0 3x3 kernel) is used rounded to bfloat16
while the trained master copy and the biases stay in higher precision, and in
the backward pass the gradient reaching each feature map is rounded to
bfloat16 before it enters the convolutions' adjoints.  The gradient of a
rounded weight is passed to its master copy unchanged (straight-through).
All arithmetic here is float64.  ``round_bf16=False`` removes every rounding
(used by the finite-difference pin).

Training target: pairs (image, plain-overfit latents and decoder parameters);
the loss of one image is mean((y - y*)^2) over all latents plus
mean((theta - theta*)^2) over the decoder parameters; a mini-batch loss is
the mean over its images.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_CH = 32          # trunk width
N_CONV = 4         # stride-2 trunk layers
N_LEVELS = 7       # latent grids produced


# ------------------------------------------------------------- bfloat16

def bf16(a):
    """Round to the nearest bfloat16 value (8 significant bits, ties to
    even, the exponent range of binary32), returned as float64."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = (a != 0) & np.isfinite(a)
    m, e = np.frexp(a[nz])                   # a = m 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)                  # below 2^-126: the subnormal spacing 2^-133
    scale = np.ldexp(1.0, 8 - e)             # 8 significant bits
    out[nz] = np.rint(a[nz] * scale) / scale
    out[~np.isfinite(a)] = a[~np.isfinite(a)]
    return out


# ------------------------------------------------------------- parameters

@dataclass(frozen=True)
class WarmLayout:
    """Offsets of the packed master parameters.

    conv k (k = 1..4): W_k [32][3][3][C_in] (out, ky, kx, in), then b_k [32];
    head level 0: V_0 [32], beta_0, K_0 [3][3][3] (ky, kx, colour);
    head level l = 1..6: V_l [32], beta_l;
    decoder-parameter head: P [n_theta][32], then pi [n_theta].
    """
    n_theta: int

    def conv(self, k):
        cin = 3 if k == 1 else N_CH
        off = 0
        for j in range(1, k):
            off += N_CH * 9 * (3 if j == 1 else N_CH) + N_CH
        return off, (N_CH, 3, 3, cin)

    @property
    def heads(self):
        off, shape = self.conv(N_CONV)
        return off + int(np.prod(shape)) + N_CH

    def head(self, l):
        """Offset of level l's head block (level 0: 60 values, others 33)."""
        return self.heads if l == 0 else self.heads + 60 + 33 * (l - 1)

    @property
    def ptheta(self):
        return self.head(N_LEVELS - 1) + 33

    @property
    def size(self):
        return self.ptheta + self.n_theta * N_CH + self.n_theta


def unpack(net, n_theta):
    lay = WarmLayout(n_theta)
    net = np.asarray(net, np.float64)
    p = {}
    for k in range(1, N_CONV + 1):
        off, shape = lay.conv(k)
        n = int(np.prod(shape))
        p[f"W{k}"] = net[off:off + n].reshape(shape)
        p[f"b{k}"] = net[off + n:off + n + N_CH]
    for l in range(N_LEVELS):
        o = lay.head(l)
        p[f"V{l}"] = net[o:o + N_CH]
        p[f"beta{l}"] = net[o + N_CH]
    o0 = lay.head(0) + N_CH + 1
    p["K0"] = net[o0:o0 + 27].reshape(3, 3, 3)
    o = lay.ptheta
    p["P"] = net[o:o + n_theta * N_CH].reshape(n_theta, N_CH)
    p["pi"] = net[o + n_theta * N_CH:o + n_theta * N_CH + n_theta]
    return p


def pack(p, n_theta):
    lay = WarmLayout(n_theta)
    net = np.zeros(lay.size)
    for k in range(1, N_CONV + 1):
        off, shape = lay.conv(k)
        n = int(np.prod(shape))
        net[off:off + n] = np.ravel(p[f"W{k}"])
        net[off + n:off + n + N_CH] = p[f"b{k}"]
    for l in range(N_LEVELS):
        o = lay.head(l)
        net[o:o + N_CH] = p[f"V{l}"]
        net[o + N_CH] = p[f"beta{l}"]
    o0 = lay.head(0) + N_CH + 1
    net[o0:o0 + 27] = np.ravel(p["K0"])
    o = lay.ptheta
    net[o:o + n_theta * N_CH] = np.ravel(p["P"])
    net[o + n_theta * N_CH:o + n_theta * N_CH + n_theta] = p["pi"]
    return net


# ------------------------------------------------------------- layers

def conv3x3_s2(f, W, b):
    """Pre-activation of a 3x3, stride-2, zero-padding-1 convolution.
    f [C_in][h][w] (h, w even), W [C_out][3][3][C_in] -> [C_out][h/2][w/2];
    output (i, j) reads input (2i + ky - 1, 2j + kx - 1)."""
    cin, h, w = f.shape
    ho, wo = h // 2, w // 2
    fp = np.pad(f, ((0, 0), (1, 1), (1, 1)))
    out = np.broadcast_to(np.asarray(b, np.float64)[:, None, None], (W.shape[0], ho, wo)).copy()
    for ky in range(3):
        for kx in range(3):
            patch = fp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2]
            out += np.einsum("oc,chw->ohw", W[:, ky, kx, :], patch)
    return out


def conv3x3_s2_adjoint(f, W, dpre):
    """Gradients of conv3x3_s2 for the output gradient dpre:
    (d input, d W, d b)."""
    cin, h, w = f.shape
    ho, wo = h // 2, w // 2
    fp = np.pad(f, ((0, 0), (1, 1), (1, 1)))
    dfp = np.zeros_like(fp)
    dW = np.zeros_like(W, dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = fp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2]
            dW[:, ky, kx, :] = np.einsum("ohw,chw->oc", dpre, patch)
            dfp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2] += np.einsum("oc,ohw->chw", W[:, ky, kx, :], dpre)
    return dfp[:, 1:-1, 1:-1], dW, dpre.sum(axis=(1, 2))


def conv3x3_s1_single(x, K):
    """One-output 3x3 convolution, stride 1, zero padding 1:
    x [3][H][W], K [3][3][3] (ky, kx, colour) -> [H][W]."""
    c, h, w = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((h, w))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("c,chw->hw", K[ky, kx], xp[:, ky:ky + h, kx:kx + w])
    return out


def avg_pool(f, k):
    c, h, w = f.shape
    return f.reshape(c, h // k, k, w // k, k).mean(axis=(2, 4))


def _r(round_bf16):
    return bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))


def forward(x, net, n_theta, round_bf16=True):
    """Warm-start prediction for one image x [3][H][W] (H, W multiples of 64).
    Returns dict(y=[7 grids], theta, f=[x~, f_1..f_4], params=rounded weights)."""
    R = _r(round_bf16)
    p = unpack(net, n_theta)
    q = {k: (R(v) if k[0] in "WVKP" else np.asarray(v, np.float64)) for k, v in p.items()}
    f = [R(x)]
    for k in range(1, N_CONV + 1):
        pre = conv3x3_s2(f[-1], q[f"W{k}"], q[f"b{k}"])
        f.append(R(np.maximum(pre, 0.0)))
    y = [None] * N_LEVELS
    for l in range(1, 5):
        y[l] = np.einsum("c,chw->hw", q[f"V{l}"], f[l]) + q[f"beta{l}"]
    y[5] = np.einsum("c,chw->hw", q["V5"], avg_pool(f[4], 2)) + q["beta5"]
    y[6] = np.einsum("c,chw->hw", q["V6"], avg_pool(f[4], 4)) + q["beta6"]
    g = np.einsum("c,chw->hw", q["V0"], f[1])
    y[0] = conv3x3_s1_single(f[0], q["K0"]) + q["beta0"] + np.kron(g, np.ones((2, 2)))
    gap = f[4].mean(axis=(1, 2))
    theta = q["P"] @ gap + q["pi"]
    return dict(y=y, theta=theta, f=f, gap=gap, q=q)


def pack_levels(y):
    return np.concatenate([np.ravel(a) for a in y])


def loss(out, y_target, theta_target):
    """Regression loss of one image against its plain-overfit target."""
    yv = pack_levels(out["y"])
    return float(np.mean((yv - y_target) ** 2) + np.mean((out["theta"] - theta_target) ** 2))


def backward(x, net, n_theta, y_target, theta_target, round_bf16=True, weight=1.0):
    """Loss of one image (times weight) and its gradient with respect to the
    packed master parameters (hand-written adjoint of forward)."""
    out = forward(x, net, n_theta, round_bf16)
    yv = pack_levels(out["y"])
    L = weight * loss(out, y_target, theta_target)
    dyv = weight * 2.0 * (yv - y_target) / yv.size
    dth = weight * 2.0 * (out["theta"] - theta_target) / n_theta
    return L, adjoint(out, n_theta, dyv, dth, round_bf16)


def backward_from_grads(x, net, n_theta, dy_packed, dtheta, round_bf16=True):
    """Gradient with respect to the packed master parameters of an outer loss
    whose gradients with respect to the outputs (packed latents, decoder
    parameters) are given."""
    out = forward(x, net, n_theta, round_bf16)
    return adjoint(out, n_theta, np.asarray(dy_packed, np.float64), np.asarray(dtheta, np.float64), round_bf16)


def adjoint(out, n_theta, dyv, dth, round_bf16=True):
    """Reverse pass of forward() for output gradients (dyv packed, dth)."""
    R = _r(round_bf16)
    f, q, y = out["f"], out["q"], out["y"]
    dy, o = [], 0
    for a in y:
        dy.append(dyv[o:o + a.size].reshape(a.shape))
        o += a.size
    g = {}
    # decoder-parameter head
    g["P"] = np.outer(dth, out["gap"])
    g["pi"] = dth
    h4, w4 = f[4].shape[1:]
    df = [None] * (N_CONV + 1)
    df[4] = np.broadcast_to((q["P"].T @ dth)[:, None, None] / (h4 * w4), f[4].shape).copy()
    # latent heads on f_4 (levels 4, 5, 6)
    for l, k in ((4, 1), (5, 2), (6, 4)):
        src = f[4] if k == 1 else avg_pool(f[4], k)
        g[f"V{l}"] = np.einsum("hw,chw->c", dy[l], src)
        g[f"beta{l}"] = dy[l].sum()
        up = dy[l] if k == 1 else np.kron(dy[l], np.ones((k, k))) / (k * k)
        df[4] += q[f"V{l}"][:, None, None] * up[None]
    # levels 1..3 and the level-0 path through f_1
    for l in (1, 2, 3):
        g[f"V{l}"] = np.einsum("hw,chw->c", dy[l], f[l])
        g[f"beta{l}"] = dy[l].sum()
    dg = dy[0].reshape(dy[0].shape[0] // 2, 2, dy[0].shape[1] // 2, 2).sum(axis=(1, 3))
    g["V0"] = np.einsum("hw,chw->c", dg, f[1])
    g["beta0"] = dy[0].sum()
    xp = np.pad(f[0], ((0, 0), (1, 1), (1, 1)))
    H, W = dy[0].shape
    g["K0"] = np.zeros((3, 3, 3))
    for ky in range(3):
        for kx in range(3):
            g["K0"][ky, kx] = np.einsum("hw,chw->c", dy[0], xp[:, ky:ky + H, kx:kx + W])
    # trunk, deepest layer first
    for k in range(N_CONV, 0, -1):
        if k < N_CONV:
            df[k] = df[k] + q[f"V{k}"][:, None, None] * dy[k][None]
            if k == 1:
                df[k] = df[k] + q["V0"][:, None, None] * dg[None]
        dpre = R(df[k] * (f[k] > 0))
        dfin, g[f"W{k}"], g[f"b{k}"] = conv3x3_s2_adjoint(f[k - 1], q[f"W{k}"], dpre)
        if k > 1:
            df[k - 1] = dfin
    return pack(g, n_theta)


def batch_backward(xs, net, n_theta, ys, thetas, round_bf16=True):
    """Mean loss over a mini-batch and its gradient."""
    B = len(xs)
    Ltot, gtot = 0.0, np.zeros(WarmLayout(n_theta).size)
    for x, yt, tt in zip(xs, ys, thetas):
        L, gr = backward(x, net, n_theta, yt, tt, round_bf16, weight=1.0 / B)
        Ltot += L
        gtot += gr
    return Ltot, gtot
