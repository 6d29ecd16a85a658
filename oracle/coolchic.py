"""Plain float64 NumPy definition of the Cool-chic rate-distortion pass.

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests, the smoke
check and the CPU-baseline leg of the benchmark may call this module.

What is computed, with the passage each part follows (Blard et al.,
"Overfitted image coding at reduced complexity"):

* Section II "Decoding": L latent grids y_l of size H/2^l x W/2^l; an
  auto-regressive model (ARM) f_psi, an MLP over neighbouring latents, gives
  the probability of each latent; a linear upsampling f_upsilon and a
  synthesis f_theta turn the grids into the decoded image.
* Section II "Encoding", Eq. (1): loss = D(x, x_hat) + lambda * R(y_hat), with D
  the mean-squared error and R = -log2 p_psi(y_hat); y_hat = Q(y) is optimised
  through a differentiable proxy of Q.
* Table I: layer shapes (InFeat-OutFeat-Layer-Kernel), residual layers
  (suffix R), stride-2 transposed convolutions, ReLU after every layer except
  the last one of each module.
* Section IV-A, Eq. (2): one training iteration is one forward and one
  backward pass; the backward computes the gradient with respect to the layer
  weights and to the layer inputs.

Readings where the paper is silent (each is listed in the design doc):
the probability model is a Laplace distribution whose mean and log-scale are
the two ARM outputs, with the scale clamped to [0.01, 100] and the rate of a
latent the -log2 of the Laplace mass over [y_hat - 1/2, y_hat + 1/2]; the
context is the C causal neighbours nearest in Euclidean distance inside a 7x7
window (ties broken in raster order), zero outside the grid, same level only,
one ARM shared by all levels; the upsampler applies, per level step, a
separable 8-tap stride-2 transposed convolution with replicate (edge-clamp)
borders; the synthesis 3x3 convolutions use replicate borders; the rate is
normalised by H*W (bits per pixel) and the distortion is the mean over 3*H*W.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

LN2 = math.log(2.0)
S_MIN = math.log(0.01)   # log-scale clamp of the Laplace scale b (reading, see above)
S_MAX = math.log(100.0)

__all__ = [
    "Arch", "TINY", "FULL", "LOW", "FD16", "TABLE1", "param_sizes", "unpack", "pack",
    "table1_param_count", "mac_per_pixel", "level_shapes", "split_levels",
    "quantise", "quantise_grad", "soft_round", "soft_round_grad", "context_offsets", "gather_context", "arm_forward", "laplace_mass",
    "rate_bits", "rate_grads", "log_laplace_mass", "tconv1d", "tconv1d_adjoint", "upsample2x",
    "tconv2d", "tconv2d_adjoint", "upsample_step",
    "upsample_pyramid", "conv3x3_replicate", "synthesis", "forward", "backward",
    "adam_step", "S_MIN", "S_MAX", "param_rate_bits", "quantize_params", "PARAM_B_MIN",
]


@dataclass(frozen=True)
class Arch:
    """Decoder architecture (Table I notation).

    n_levels   : L, number of latent grids (Section II).
    arm_ctx    : C, ARM input width = number of causal neighbours; the hidden
                 LinR layers are C -> C (residual needs equal widths).
    arm_layers : number of hidden C-C-LinR layers before the C-2-Lin output.
    ups_taps   : K, taps of each stride-2 transposed convolution (4 or 8).
    syn_hidden : width of the first 1x1 synthesis layer (L -> syn_hidden).
    syn_res    : number of 3-3-ConvR-3 residual 3x3 convolutions.
    ups_shared : False: each upsampling step has its own separable kernel (a
                 vertical and a horizontal K-tap filter); True: Table I's
                 "1-1-TConv-K", one non-separable K x K kernel shared by every
                 step (K*K parameters).
    """
    n_levels: int = 7
    arm_ctx: int = 24
    arm_layers: int = 2
    ups_taps: int = 8
    syn_hidden: int = 40
    syn_res: int = 2
    ups_shared: bool = False


# Table I's four decoders (300 / 545 / 1079 / 2300 MAC per pixel)
TABLE1 = {300: Arch(7, 8, 1, 4, 8, 1, True), 545: Arch(7, 8, 2, 4, 16, 2, True),
          1079: Arch(7, 16, 2, 4, 16, 2, True), 2300: Arch(7, 24, 2, 8, 40, 2, True)}
TINY = Arch(7, 8, 2, 8, 16, 1)    # 64x64 small instance
FULL = Arch(7, 24, 2, 8, 40, 2)   # Table I 2300 row with a separable per-level upsampler
LOW = Arch(7, 8, 2, 8, 16, 1)     # low-complexity decoder
FD16 = Arch(5, 8, 2, 8, 16, 1)    # 16x16 finite-difference instance (5 levels)


# ----------------------------------------------------------------------------
# parameter layout and counting
# ----------------------------------------------------------------------------
def param_sizes(arch: Arch):
    """(n_arm, n_ups, n_syn): every ARM and synthesis layer has a bias
    (Table I parameter counts), the upsampler has none."""
    C, L, Hs, K = arch.arm_ctx, arch.n_levels, arch.syn_hidden, arch.ups_taps
    n_arm = arch.arm_layers * (C * C + C) + 2 * C + 2
    n_ups = K * K if arch.ups_shared else (L - 1) * 2 * K
    n_syn = Hs * L + Hs + 3 * Hs + 3 + arch.syn_res * (3 * 3 * 3 * 3 + 3)
    return n_arm, n_ups, n_syn


def unpack(arch: Arch, arm_w, ups_w, syn_w):
    """Split the three flat parameter vectors into named float64 arrays.

    ARM  : for each hidden layer (W [C][C] (out, in), b [C]); then Wo [2][C]
           (row 0 = mean, row 1 = log-scale) and bo [2].
    UPS  : separable: [L-1][2][K]; index s produces level s from level s+1;
           [0] holds the vertical taps, [1] the horizontal taps.  Shared:
           [K][K] (ky, kx), one kernel for every step.
    SYN  : W1 [Hs][L], b1 [Hs], W2 [3][Hs], b2 [3]; per residual conv
           W [3][3][3][3] (out, in, ky, kx), b [3].
    """
    C, L, Hs, K = arch.arm_ctx, arch.n_levels, arch.syn_hidden, arch.ups_taps
    a = np.asarray(arm_w, dtype=np.float64)
    n_arm, n_ups, n_syn = param_sizes(arch)
    assert a.size == n_arm and np.size(ups_w) == n_ups and np.size(syn_w) == n_syn
    o = 0
    hidden = []
    for _ in range(arch.arm_layers):
        W = a[o:o + C * C].reshape(C, C); o += C * C
        b = a[o:o + C]; o += C
        hidden.append((W, b))
    Wo = a[o:o + 2 * C].reshape(2, C); o += 2 * C
    bo = a[o:o + 2]; o += 2
    ups = np.asarray(ups_w, dtype=np.float64).reshape((K, K) if arch.ups_shared else (L - 1, 2, K))
    s = np.asarray(syn_w, dtype=np.float64)
    o = 0
    W1 = s[o:o + Hs * L].reshape(Hs, L); o += Hs * L
    b1 = s[o:o + Hs]; o += Hs
    W2 = s[o:o + 3 * Hs].reshape(3, Hs); o += 3 * Hs
    b2 = s[o:o + 3]; o += 3
    res = []
    for _ in range(arch.syn_res):
        Wr = s[o:o + 81].reshape(3, 3, 3, 3); o += 81
        br = s[o:o + 3]; o += 3
        res.append((Wr, br))
    return dict(hidden=hidden, Wo=Wo, bo=bo, ups=ups, W1=W1, b1=b1, W2=W2, b2=b2, res=res)


def pack(arch: Arch, P):
    """Inverse of :func:`unpack` (used for gradients): returns (arm, ups, syn)."""
    arm = []
    for (W, b) in P["hidden"]:
        arm += [np.ravel(W), np.ravel(b)]
    arm += [np.ravel(P["Wo"]), np.ravel(P["bo"])]
    syn = [np.ravel(P["W1"]), np.ravel(P["b1"]), np.ravel(P["W2"]), np.ravel(P["b2"])]
    for (Wr, br) in P["res"]:
        syn += [np.ravel(Wr), np.ravel(br)]
    return np.concatenate(arm), np.ravel(P["ups"]).copy(), np.concatenate(syn)


def table1_param_count(arm_width, arm_hidden, tconv_k, syn_hidden, syn_res, n_levels=7):
    """Parameter count of a Table I decoder: ARM (arm_hidden residual
    width-width LinR layers, then width-2 Lin), one shared 1-1 TConv-K kernel
    (K*K taps, no bias), synthesis L-Hs Conv-1, Hs-3 Conv-1 and syn_res 3-3
    ConvR-3, every ARM / synthesis layer with a bias.  Returns
    (arm, ups, syn, total)."""
    C = arm_width
    arm = arm_hidden * (C * C + C) + (2 * C + 2)
    ups = tconv_k * tconv_k
    syn = (n_levels * syn_hidden + syn_hidden) + (syn_hidden * 3 + 3) + syn_res * (81 + 3)
    return arm, ups, syn, arm + ups + syn


def mac_per_pixel(arm_width, arm_hidden, tconv_k, syn_hidden, syn_res, H=512, W=768,
                  n_levels=7, separable=False):
    """Decoder multiplications per pixel (Section III-A complexity in MAC/pixel).

    ARM: arm_hidden * C^2 + 2C MAC per latent, times N_lat / N_px.
    Upsampling: the grid of level l is brought to full resolution through the
    levels below it, so sum_s (L-1-s) * N_s outputs are produced per image; a
    shared K x K stride-2 kernel costs K^2/4 MAC per output, a separable one
    K/4 (vertical half-resolution pass) + K/2 (horizontal pass).
    Synthesis: L*Hs + Hs*3 + syn_res*81 MAC per pixel.
    Returns (arm, ups, syn, total)."""
    shapes = level_shapes(H, W, n_levels)
    n_lat = sum(h * w for h, w in shapes)
    n_px = H * W
    C = arm_width
    arm = (arm_hidden * C * C + 2 * C) * n_lat / n_px
    outs = sum((n_levels - 1 - s) * shapes[s][0] * shapes[s][1] for s in range(n_levels - 1)) / n_px
    per_out = (tconv_k / 4 + tconv_k / 2) if separable else tconv_k * tconv_k / 4
    ups = per_out * outs
    syn = n_levels * syn_hidden + syn_hidden * 3 + syn_res * 81
    return arm, ups, syn, arm + ups + syn


# ----------------------------------------------------------------------------
# latents and quantisation
# ----------------------------------------------------------------------------
def level_shapes(H, W, L):
    """Grid l has H/2^l x W/2^l latents (Section II)."""
    return [(H >> l, W >> l) for l in range(L)]


def split_levels(vec, H, W, L):
    """Packed level-major row-major pyramid -> list of 2-D float64 arrays."""
    out, o = [], 0
    v = np.asarray(vec, dtype=np.float64)
    for (h, w) in level_shapes(H, W, L):
        out.append(v[o:o + h * w].reshape(h, w))
        o += h * w
    assert o == v.size
    return out


def soft_round(x, alpha):
    """Soft rounding (Agustsson & Theis, "Universally quantized neural
    compression", 2020): floor(x) + 1/2 + tanh(alpha r) / (2 tanh(alpha / 2))
    with r = x - floor(x) - 1/2; it passes through every integer and half
    integer, tends to rounding as alpha grows and to the identity as alpha
    goes to 0."""
    x = np.asarray(x, dtype=np.float64)
    fl = np.floor(x)
    return fl + 0.5 + np.tanh(alpha * (x - fl - 0.5)) / (2.0 * np.tanh(alpha / 2.0))


def soft_round_grad(x, alpha):
    """d soft_round / dx = alpha (1 - tanh^2(alpha r)) / (2 tanh(alpha / 2))."""
    x = np.asarray(x, dtype=np.float64)
    t = np.tanh(alpha * (x - np.floor(x) - 0.5))
    return alpha * (1.0 - t * t) / (2.0 * np.tanh(alpha / 2.0))


def quantise(y, u=None, alpha=None):
    """y_hat = Q(y) (Section II "Encoding").  Without noise: round to the
    nearest integer, ties to even; its gradient is taken as the identity
    (straight-through).  With noise u in [-1/2, 1/2): y_hat = y + u, the
    additive-noise proxy, whose gradient is the identity too.  With alpha
    (the proxy C3 uses, cited in Section II): y_hat = s(s(y) + u) with s the
    soft rounding of sharpness alpha; its gradient is s'(s(y) + u) s'(y)."""
    y = np.asarray(y, dtype=np.float64)
    if alpha is not None:
        return soft_round(soft_round(y, alpha) + np.asarray(u, dtype=np.float64), alpha)
    if u is None:
        return np.rint(y)
    return y + np.asarray(u, dtype=np.float64)


def quantise_grad(y, u, alpha):
    """dy_hat/dy of the soft proxy (1 for the other two)."""
    y = np.asarray(y, dtype=np.float64)
    if alpha is None:
        return np.ones_like(y)
    return soft_round_grad(soft_round(y, alpha) + np.asarray(u, dtype=np.float64), alpha) * soft_round_grad(y, alpha)


# ----------------------------------------------------------------------------
# ARM: causal context, MLP, Laplace rate
# ----------------------------------------------------------------------------
def context_offsets(C):
    """The C causal neighbours (dy, dx) of a latent: all positions of a 7x7
    window that precede it in raster order, taken by increasing Euclidean
    distance with ties in raster order, then listed in raster order.  C = 24
    is the whole causal half of the window."""
    cands = [(dy, dx) for dy in range(-3, 1) for dx in range(-3, 4) if dy < 0 or dx < 0]
    cands.sort(key=lambda o: (o[0] * o[0] + o[1] * o[1], o[0], o[1]))
    if C > len(cands):
        raise ValueError("context larger than the causal 7x7 window")
    return sorted(cands[:C])


def gather_context(level, offsets):
    """Context matrix [h*w][C]: c_k = y_hat[i+dy_k, j+dx_k], zero outside the
    grid (Section II: the ARM is conditioned on neighbouring values)."""
    h, w = level.shape
    P = np.zeros((h + 6, w + 6))
    P[3:3 + h, 3:3 + w] = level
    ctx = np.empty((h * w, len(offsets)))
    for k, (dy, dx) in enumerate(offsets):
        ctx[:, k] = P[3 + dy:3 + dy + h, 3 + dx:3 + dx + w].ravel()
    return ctx


def arm_forward(ctx, P):
    """ARM MLP f_psi (Table I "C-C-LinR, C-2-Lin"): h <- ReLU(W h + b + h) per
    hidden layer, then (mu, s) = Wo h + bo.  Returns mu, s and the hidden
    activations (pre-activations kept for the adjoint)."""
    h = ctx
    cache = [h]
    for (W, b) in P["hidden"]:
        pre = h @ W.T + b + h
        h = np.maximum(pre, 0.0)
        cache.append(h)
    out = h @ P["Wo"].T + P["bo"]
    return out[:, 0], out[:, 1], cache


def _laplace_cdf(x, mu, b):
    z = (x - mu) / b
    neg = z < 0
    out = np.empty_like(z)
    out[neg] = 0.5 * np.exp(z[neg])
    out[~neg] = 1.0 - 0.5 * np.exp(-z[~neg])
    return out


def _laplace_sf(x, mu, b):
    """1 - F(x), for x >= mu."""
    return 0.5 * np.exp(-(x - mu) / b)


def laplace_mass(yq, mu, b):
    """P(y_hat) = F(y_hat + 1/2) - F(y_hat - 1/2), F the Laplace(mu, b) CDF.
    In the right tail the same difference is taken as S(y_hat - 1/2) -
    S(y_hat + 1/2) with S = 1 - F, which avoids subtracting two numbers near 1."""
    yq, mu, b = np.broadcast_arrays(np.asarray(yq, float), np.asarray(mu, float), np.asarray(b, float))
    lo, hi = yq - 0.5, yq + 0.5
    right = lo >= mu
    P = np.empty(yq.shape)
    P[right] = _laplace_sf(lo[right], mu[right], b[right]) - _laplace_sf(hi[right], mu[right], b[right])
    nr = ~right
    P[nr] = _laplace_cdf(hi[nr], mu[nr], b[nr]) - _laplace_cdf(lo[nr], mu[nr], b[nr])
    return P


TAIL_LOG_BELOW = 1e-280   # masses below this are taken in log space


def log_laplace_mass(yq, mu, b):
    """Natural log of :func:`laplace_mass`.  Where the mass is too small for
    float64 (far tails), the same difference is factored before taking the
    log: both bounds on one side of mu give
    F(hi) - F(lo) = (1/2) e^{-dist/b} (1 - e^{-1/b}), dist the distance from mu
    to the nearer bound."""
    yq, mu, b = np.broadcast_arrays(np.asarray(yq, float), np.asarray(mu, float), np.asarray(b, float))
    P = laplace_mass(yq, mu, b)
    out = np.empty(P.shape)
    ok = P > TAIL_LOG_BELOW
    out[ok] = np.log(P[ok])
    t = ~ok
    if t.any():
        lo, hi = yq[t] - 0.5, yq[t] + 0.5
        m, bb = mu[t], b[t]
        dist = np.where(lo >= m, lo - m, m - hi)
        assert np.all(dist >= 0), "a mass that straddles the mean cannot underflow"
        out[t] = -dist / bb - math.log(2.0) + np.log1p(-np.exp(-1.0 / bb))
    return out


def rate_bits(yq, mu, s):
    """Rate of each latent in bits, -log2 p(y_hat) (Eq. (1)), with the Laplace
    scale b = exp(clamp(s, ln 0.01, ln 100))."""
    b = np.exp(np.clip(np.asarray(s, float), S_MIN, S_MAX))
    return -log_laplace_mass(yq, mu, b) / LN2


def rate_grads(yq, mu, s):
    """(dr/dy_hat, dr/dmu, dr/ds) of r = -log2 P, from the derivatives of the
    CDF difference: dP/dy_hat = f(hi) - f(lo) with f the Laplace density,
    dP/dmu = -dP/dy_hat, dP/db = -[(hi-mu) f(hi) - (lo-mu) f(lo)] / b, and
    db/ds = b inside the clamp range (bounds included), 0 outside.  The
    ratios f / P are formed as exp(log f - log P) so that tails stay finite."""
    yq, mu, s = (np.asarray(a, float) for a in (yq, mu, s))
    b = np.exp(np.clip(s, S_MIN, S_MAX))
    lo, hi = yq - 0.5, yq + 0.5
    logP = log_laplace_mass(yq, mu, b)
    fr = lambda x: np.exp(-np.abs(x - mu) / b - np.log(2.0 * b) - logP)  # noqa: E731  f(x) / P
    dP_dy = fr(hi) - fr(lo)
    dP_db = -((hi - mu) * fr(hi) - (lo - mu) * fr(lo)) / b
    k = -1.0 / LN2
    inside = (s >= S_MIN) & (s <= S_MAX)
    return k * dP_dy, -k * dP_dy, k * dP_db * b * inside


# ----------------------------------------------------------------------------
# upsampling f_upsilon
# ----------------------------------------------------------------------------
def _tconv_index(n, K):
    p = K // 2 - 1
    js = np.arange(2 * n)
    taps = []
    for k in range(K):
        m = (js + p - k) % 2 == 0
        idx = np.clip((js[m] + p - k) // 2, 0, n - 1)
        taps.append((k, js[m], idx))
    return taps


def tconv1d(a, w, axis):
    """1-D stride-2 transposed convolution with K taps (Table I "TConv"):
    out[j] = sum over k with (j + p - k) even of w[k] * a[clamp((j + p - k)/2)],
    p = K/2 - 1, output length 2n; input indices outside [0, n) are clamped
    (replicate border)."""
    a = np.moveaxis(np.asarray(a, float), axis, -1)
    n = a.shape[-1]
    out = np.zeros(a.shape[:-1] + (2 * n,))
    for (k, js, idx) in _tconv_index(n, len(w)):
        out[..., js] += w[k] * a[..., idx]
    return np.moveaxis(out, -1, axis)


def tconv1d_adjoint(g_out, a, w, axis):
    """Adjoint of :func:`tconv1d`: returns (dL/da, dL/dw)."""
    g = np.moveaxis(np.asarray(g_out, float), axis, -1)
    a = np.moveaxis(np.asarray(a, float), axis, -1)
    n = a.shape[-1]
    ga = np.zeros(a.shape)
    gw = np.zeros(len(w))
    for (k, js, idx) in _tconv_index(n, len(w)):
        gk = g[..., js]
        np.add.at(ga, (Ellipsis, idx), w[k] * gk)
        gw[k] = np.sum(gk * a[..., idx])
    return np.moveaxis(ga, -1, axis), gw


def upsample2x(stack, v, h):
    """One 2x step: vertical pass with taps v, then horizontal pass with taps h,
    applied to every channel of stack [C][n_y][n_x]."""
    return tconv1d(tconv1d(stack, v, axis=-2), h, axis=-1)


def tconv2d(a, Wk):
    """2-D stride-2 transposed convolution with one K x K kernel (Table I
    "1-1-TConv-K"), applied to every channel of a [C][n_y][n_x]:
    out[i, j] = sum over (ky, kx) with (i + p - ky) and (j + p - kx) even of
    Wk[ky, kx] * a[clamp((i + p - ky)/2), clamp((j + p - kx)/2)], p = K/2 - 1,
    replicate border as in the 1-D case."""
    a = np.asarray(a, float)
    K = Wk.shape[0]
    ny, nx = a.shape[-2:]
    out = np.zeros(a.shape[:-2] + (2 * ny, 2 * nx))
    for (ky, rows, ridx) in _tconv_index(ny, K):
        for (kx, cols, cidx) in _tconv_index(nx, K):
            out[..., rows[:, None], cols[None, :]] += Wk[ky, kx] * a[..., ridx[:, None], cidx[None, :]]
    return out


def tconv2d_adjoint(g_out, a, Wk):
    """Adjoint of :func:`tconv2d`: returns (dL/da, dL/dWk)."""
    g = np.asarray(g_out, float)
    a = np.asarray(a, float)
    K = Wk.shape[0]
    ny, nx = a.shape[-2:]
    ga = np.zeros(a.shape)
    gW = np.zeros((K, K))
    for (ky, rows, ridx) in _tconv_index(ny, K):
        for (kx, cols, cidx) in _tconv_index(nx, K):
            gk = g[..., rows[:, None], cols[None, :]]
            np.add.at(ga, (Ellipsis, ridx[:, None], cidx[None, :]), Wk[ky, kx] * gk)
            gW[ky, kx] = np.sum(gk * a[..., ridx[:, None], cidx[None, :]])
    return ga, gW


def upsample_step(stack, ups, s):
    """U_s: the separable kernel of step s (ups [L-1][2][K]) or the shared
    K x K kernel (ups [K][K])."""
    if ups.ndim == 2:
        return tconv2d(stack, ups)
    return upsample2x(stack, ups[s, 0], ups[s, 1])


def upsample_pyramid(levels, ups):
    """Bring every grid to full resolution (Section II f_upsilon): stack_{L-1}
    = y_hat_{L-1}; stack_s = [y_hat_s, U_s(stack_{s+1})] for s = L-2 .. 0.
    Returns z = stack_0 [L][H][W] (channel l is level l) and all stacks."""
    L = len(levels)
    stack = levels[L - 1][None]
    stacks = {L - 1: stack}
    for s in range(L - 2, -1, -1):
        up = upsample_step(stack, ups, s)
        stack = np.concatenate([levels[s][None], up], axis=0)
        stacks[s] = stack
    return stack, stacks


# ----------------------------------------------------------------------------
# synthesis f_theta
# ----------------------------------------------------------------------------
def conv3x3_replicate(t, W, b):
    """3x3 cross-correlation with replicate borders:
    out[o,i,j] = sum_c sum_{dy,dx} W[o,c,dy+1,dx+1] t[c, clamp(i+dy), clamp(j+dx)] + b[o]."""
    C, H, Wd = t.shape
    tp = np.pad(t, ((0, 0), (1, 1), (1, 1)), mode="edge")
    out = np.zeros((W.shape[0], H, Wd)) + b[:, None, None]
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,chw->ohw", W[:, :, ky, kx], tp[:, ky:ky + H, kx:kx + Wd])
    return out


def synthesis(z, P):
    """Synthesis f_theta (Table I): L-Hs Conv-1 + ReLU, Hs-3 Conv-1 + ReLU, then
    residual 3-3-ConvR-3 layers t <- phi(t + conv(t) + b), phi = ReLU except
    after the last layer.  Returns x_hat and the intermediates."""
    pre_a = np.einsum("fl,lhw->fhw", P["W1"], z) + P["b1"][:, None, None]
    a = np.maximum(pre_a, 0.0)
    pre_t = np.einsum("cf,fhw->chw", P["W2"], a) + P["b2"][:, None, None]
    t = np.maximum(pre_t, 0.0)
    ts, pres = [t], []
    n = len(P["res"])
    for r, (Wr, br) in enumerate(P["res"]):
        pre = t + conv3x3_replicate(t, Wr, br)
        pres.append(pre)
        t = np.maximum(pre, 0.0) if r < n - 1 else pre
        ts.append(t)
    return t, dict(pre_a=pre_a, a=a, pre_t=pre_t, ts=ts, pres=pres)


# ----------------------------------------------------------------------------
# the rate-distortion pass and its gradient
# ----------------------------------------------------------------------------
def _as64(*arrs):
    return [None if a is None else np.asarray(a, dtype=np.float64) for a in arrs]


def forward(arch: Arch, img, y, arm_w, ups_w, syn_w, lam, u=None, soft_alpha=None):
    """Eq. (1): loss = D + lambda * R / (H W), D = mean over 3HW of
    (x_hat - x)^2, R = sum of the per-latent rates in bits.  Returns a dict
    with loss, D, R, the per-latent rate map, y_hat, x_hat, mu and s.
    soft_alpha: the soft-rounding proxy of :func:`quantise` (u required)."""
    img, y, u = _as64(img, y, u)
    _, H, W = img.shape
    L = arch.n_levels
    P = unpack(arch, arm_w, ups_w, syn_w)
    yq = quantise(y, u, soft_alpha)
    levels = split_levels(yq, H, W, L)
    offs = context_offsets(arch.arm_ctx)
    mus, ss = [], []
    for lv in levels:
        mu, s, _ = arm_forward(gather_context(lv, offs), P)
        mus.append(mu)
        ss.append(s)
    mu = np.concatenate(mus)
    s = np.concatenate(ss)
    rate = rate_bits(yq, mu, s)
    R = float(np.sum(rate))
    z, _ = upsample_pyramid(levels, P["ups"])
    xhat, _ = synthesis(z, P)
    D = float(np.mean((xhat - img) ** 2))
    loss = D + lam * R / (H * W)
    return dict(loss=loss, D=D, R=R, rate=rate, yq=yq, xhat=xhat, mu=mu, s=s)


def _conv3x3_adjoint(g, t, W):
    """Adjoint of conv3x3_replicate w.r.t. its input and weights (bias: sum of g).
    The replicate border is handled by scattering into the padded frame and
    folding the frame back onto the edge rows / columns."""
    C, H, Wd = t.shape
    tp = np.pad(t, ((0, 0), (1, 1), (1, 1)), mode="edge")
    gp = np.zeros((C, H + 2, Wd + 2))
    gW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            gp[:, ky:ky + H, kx:kx + Wd] += np.einsum("oc,ohw->chw", W[:, :, ky, kx], g)
            gW[:, :, ky, kx] = np.einsum("ohw,chw->oc", g, tp[:, ky:ky + H, kx:kx + Wd])
    gp[:, 1, :] += gp[:, 0, :]
    gp[:, H, :] += gp[:, H + 1, :]
    gp[:, :, 1] += gp[:, :, 0]
    gp[:, :, Wd] += gp[:, :, Wd + 1]
    return gp[:, 1:H + 1, 1:Wd + 1], gW


def backward(arch: Arch, img, y, arm_w, ups_w, syn_w, lam, u=None, dloss=1.0, soft_alpha=None):
    """Hand-written reverse mode of :func:`forward` (Section IV-A: each layer
    returns the gradient w.r.t. its weights and w.r.t. its input).  The
    quantiser passes the gradient through unchanged (straight-through for
    rounding, exact for additive noise); the soft proxy multiplies it by its
    derivative.  ReLU'(0) = 0.  Returns the forward dict plus g_y, g_arm,
    g_ups, g_syn (flat, laid out like the inputs)."""
    img, y, u = _as64(img, y, u)
    _, H, W = img.shape
    L = arch.n_levels
    P = unpack(arch, arm_w, ups_w, syn_w)
    yq = quantise(y, u, soft_alpha)
    levels = split_levels(yq, H, W, L)
    offs = context_offsets(arch.arm_ctx)
    shapes = level_shapes(H, W, L)

    G = dict(hidden=[(np.zeros_like(Wj), np.zeros_like(bj)) for (Wj, bj) in P["hidden"]],
             Wo=np.zeros_like(P["Wo"]), bo=np.zeros_like(P["bo"]), ups=np.zeros_like(P["ups"]),
             W1=None, b1=None, W2=None, b2=None, res=[])
    g_levels = [np.zeros(sh) for sh in shapes]

    # ---- rate branch: lambda * R / (HW)
    kr = dloss * lam / (H * W)
    R = 0.0
    rates, mus, ss = [], [], []
    for l, lv in enumerate(levels):
        h, w = lv.shape
        ctx = gather_context(lv, offs)
        mu, s, cache = arm_forward(ctx, P)
        yl = lv.ravel()
        r = rate_bits(yl, mu, s)
        R += float(np.sum(r))
        rates.append(r); mus.append(mu); ss.append(s)
        d_y, d_mu, d_s = rate_grads(yl, mu, s)
        g_own = kr * d_y
        g_out = kr * np.stack([d_mu, d_s], axis=1)            # [N][2]
        hN = cache[-1]
        G["Wo"] += g_out.T @ hN
        G["bo"] += g_out.sum(0)
        gh = g_out @ P["Wo"]                                  # [N][C]
        for j in range(len(P["hidden"]) - 1, -1, -1):
            Wj, _ = P["hidden"][j]
            hin, hout = cache[j], cache[j + 1]
            gpre = gh * (hout > 0)
            G["hidden"][j][0][...] += gpre.T @ hin
            G["hidden"][j][1][...] += gpre.sum(0)
            gh = gpre @ Wj + gpre                             # residual: h_in also added
        # gh is now dL/dctx [N][C]; send each column back to its neighbour
        gpad = np.zeros((h + 6, w + 6))
        for k, (dy, dx) in enumerate(offs):
            gpad[3 + dy:3 + dy + h, 3 + dx:3 + dx + w] += gh[:, k].reshape(h, w)
        g_levels[l] += gpad[3:3 + h, 3:3 + w] + g_own.reshape(h, w)

    # ---- distortion branch
    z, stacks = upsample_pyramid(levels, P["ups"])
    xhat, c = synthesis(z, P)
    D = float(np.mean((xhat - img) ** 2))
    g_t = dloss * 2.0 * (xhat - img) / (3 * H * W)
    n_res = len(P["res"])
    g_res = [None] * n_res
    for r in range(n_res - 1, -1, -1):
        Wr, br = P["res"][r]
        pre, tin = c["pres"][r], c["ts"][r]
        gpre = g_t * (pre > 0) if r < n_res - 1 else g_t
        gin, gW = _conv3x3_adjoint(gpre, tin, Wr)
        g_res[r] = (gW, gpre.sum(axis=(1, 2)))
        g_t = gpre + gin
    gpre_t = g_t * (c["pre_t"] > 0)
    G["W2"] = np.einsum("chw,fhw->cf", gpre_t, c["a"])
    G["b2"] = gpre_t.sum(axis=(1, 2))
    g_a = np.einsum("cf,chw->fhw", P["W2"], gpre_t)
    gpre_a = g_a * (c["pre_a"] > 0)
    G["W1"] = np.einsum("fhw,lhw->fl", gpre_a, z)
    G["b1"] = gpre_a.sum(axis=(1, 2))
    g_z = np.einsum("fl,fhw->lhw", P["W1"], gpre_a)
    G["res"] = g_res
    # upsampling chain, s = 0 .. L-2: g_stack_s -> g_y_hat_s and g_stack_{s+1}
    g_stack = g_z
    for s in range(0, L - 1):
        g_levels[s] += g_stack[0]
        src = stacks[s + 1]
        if arch.ups_shared:
            g_src, gW = tconv2d_adjoint(g_stack[1:], src, P["ups"])
            G["ups"] += gW
        else:
            tmp = tconv1d(src, P["ups"][s, 0], axis=-2)
            g_tmp, gh = tconv1d_adjoint(g_stack[1:], tmp, P["ups"][s, 1], axis=-1)
            g_src, gv = tconv1d_adjoint(g_tmp, src, P["ups"][s, 0], axis=-2)
            G["ups"][s, 0] += gv
            G["ups"][s, 1] += gh
        g_stack = g_src
    g_levels[L - 1] += g_stack[0]

    g_y = np.concatenate([g.ravel() for g in g_levels]) * quantise_grad(y, u, soft_alpha)
    g_arm, g_ups, g_syn = pack(arch, G)
    rate = np.concatenate(rates)
    loss = D + lam * R / (H * W)
    return dict(loss=loss, D=D, R=R, rate=rate, yq=yq, xhat=xhat,
                mu=np.concatenate(mus), s=np.concatenate(ss),
                g_y=g_y, g_arm=g_arm, g_ups=g_ups, g_syn=g_syn)


def adam_step(theta, g, m, v, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, the optimiser the paper names for
    training): biased moments, bias correction with step t (1-based).
    Returns new (theta, m, v)."""
    theta, g, m, v = _as64(theta, g, m, v)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# quantisation of the decoder parameters (Section II: after the encoding the
# network parameters are quantised and entropy coded with an ad-hoc
# probability model)
# ----------------------------------------------------------------------------
PARAM_B_MIN = 0.01   # smallest Laplace scale of the parameter model (reading)


def param_rate_bits(q):
    """Bits of the integer vector q under the Laplace(0, b) model with b the
    mean |q| (its maximum-likelihood scale), at least PARAM_B_MIN: the sum of
    -log2 of the mass over [q - 1/2, q + 1/2]."""
    q = np.asarray(q, np.float64)
    if q.size == 0:
        return 0.0
    b = max(float(np.mean(np.abs(q))), PARAM_B_MIN)
    return float(np.sum(-log_laplace_mass(q, np.zeros_like(q), np.full_like(q, b)) / LN2))


def quantize_params(arm_w, ups_w, syn_w, step_log2):
    """Each module (ARM, upsampling, synthesis) on its own grid of step
    2^-k, k = step_log2[m]: q = rint(theta 2^k), theta_hat = q 2^-k.
    Returns (arm_hat, ups_hat, syn_hat, bits [3], q blocks)."""
    outs, bits, qs = [], [], []
    for w, k in zip((arm_w, ups_w, syn_w), step_log2):
        w = np.asarray(w, np.float64)
        q = np.rint(w * 2.0 ** k)
        outs.append(q * 2.0 ** -k)
        bits.append(param_rate_bits(q))
        qs.append(q)
    return outs[0], outs[1], outs[2], np.array(bits), qs
