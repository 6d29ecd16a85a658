"""Entropy coding of the quantised latents with the ARM's probabilities:
plain Python / NumPy definition (frequency tables in float64, the coder in
Python integers).

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the CPU-baseline leg
of the benchmark may call this module; it shares no code with the HIP library.

What is coded, with the passage each part follows (Blard et al., "Overfitted
image coding at reduced complexity"):

* Section II "Decoding": the latent grids are transmitted with an entropy
  coder driven by the auto-regressive model p_psi; p_psi gives the
  distribution of one latent from its already decoded neighbours, so a
  latent can only be decoded once its causal context is.
* Section II "Encoding": after training the latents are entropy coded with a
  range coder driven by p_psi.
* Section III-B "Fast decoder implementation": the decoder's ARM is
  sequential; the paper's CPU decoder swaps the range coder for a binary
  arithmetic coder.

Readings taken where the paper gives no detail (each is listed in the design doc):

* Coder: range-variant asymmetric numeral systems (rANS; Duda 2013) with a
  32-bit state in [2^23, 2^31), byte-wise renormalisation and 16-bit
  frequencies (7 bits of headroom between the state's lower bound and the
  frequency total, so the coding loss stays near 1e-3 bit per symbol),
  several states interleaved in one byte stream (Giesen 2014): a
  range-coding family coder whose decoder state updates run side by side.
* Probability model per latent: the Laplace distribution of the training
  rate (mean mu and log-scale s from the ARM, b = exp(clamp(s, ln 0.01,
  ln 100))) with its parameters quantised for coding, decided in float32 from
  the ARM outputs: scale index j = rint(8 (s_c - ln 0.01)), s_c the clamped
  s (a NaN taken as the upper bound), so b_j = exp(ln 0.01 + j / 8), j in
  0..74; mean offset c + f / 16 with c = floor(mu), f = rint(16 frac(mu))
  (f = 16 carries into c; mu clamped to +-2^20, a NaN taken as 0).
* Alphabet: d = y_hat - c in [-48, 48] (97 symbols) plus an escape symbol
  that lumps both tails; every symbol gets a frequency of at least 1 (the
  probability floor: 1 + floor(P (2^16 - 98)), the remainder added to the
  most frequent symbol, the first one on a tie).  An escaped latent then
  sends m + 1 = |d| - 48 as the bit length n (5 raw bits holding n - 1), the
  n - 1 bits below the leading one in chunks of at most 8 (the first chunk
  takes the remainder of n - 1 modulo 8, most significant first), and the
  sign (1 raw bit, 1 for negative).  A raw k-bit value v is the symbol with
  cumulative frequency v 2^(16-k) and frequency 2^(16-k).
* Decode order (the wavefront that makes every context available): within
  a grid with w columns and h rows, step t = 0 .. w - 1 + a (h - 1) decodes
  the latents (i, t - a i), rows ascending, where a is the smallest slope
  that puts every causal neighbour in an earlier step (a = 1 + max over
  context offsets with dy < 0 of floor(dx / -dy): 2, 3, 4 for C = 8, 16, 24).
  Level 0 forms one set of coder states, levels 1 .. L-1 (in ascending
  order) another.  A set has n = min(64, rows of its first level) states;
  row i is coded by state i mod n; the rows of one step are taken in groups
  of n consecutive rows (group g: rows g n .. g n + n - 1); a group is a
  round of its primary symbols, then rounds q = 1, 2, ... of the q-th escape
  payload symbol of the latents that have one.  In a round every state
  decodes its symbol, then the states whose value fell below 2^23 read bytes
  from the set's stream (one or two, until the value is back at 2^23 or
  above), state after state in ascending order.
* Bitstream (little-endian): b"CCR1", u32 number of sets, u32 byte count of
  each set, the final encoder state of each state of each set (u32), then
  each set's bytes.  Encoder states start at 2^23.
"""
from __future__ import annotations

import math

import numpy as np

from .coolchic import Arch, arm_forward, context_offsets, gather_context, level_shapes, split_levels, unpack

PREC = 16
TOTAL = 1 << PREC                 # frequency total of every table row
RANS_L = 1 << 23                  # lower bound of the coder state
A = 48                            # |d| <= A has a symbol of its own
NSYM = 2 * A + 2                  # 97 symbols and the escape
ESC = NSYM - 1
N_MU = 16                         # mean offsets per integer
SCALE_PER_LN = 8                  # scale indices per unit of ln b
LOG_BMIN32 = np.float32(math.log(0.01))
LOG_BMAX32 = np.float32(math.log(100.0))
N_SCALE = int(np.rint(np.float32(LOG_BMAX32 - LOG_BMIN32) * np.float32(SCALE_PER_LN))) + 1
MU_LIM = np.float32(1 << 20)
MAX_LANES = 64
MAGIC = b"CCR1"

__all__ = ["PREC", "TOTAL", "A", "NSYM", "ESC", "N_MU", "N_SCALE", "laplace_row_masses", "freq_table",
           "cum_table", "coding_decision", "escape_payload", "wavefront_slope", "decode_schedule",
           "rans_encode_rounds", "encode", "decode", "ideal_bits", "coding_params"]


# ----------------------------------------------------------------------------
# frequency tables
# ----------------------------------------------------------------------------
def scale_of(j):
    """Laplace scale b_j of scale index j (float64)."""
    return math.exp(float(LOG_BMIN32) + j / SCALE_PER_LN)


def laplace_row_masses(j, f):
    """Masses of the NSYM symbols of table row (j, f): symbol k < ESC is
    d = k - A, the Laplace(f / 16, b_j) mass over [d - 1/2, d + 1/2]; ESC is
    the mass of both tails beyond [-A - 1/2, A + 1/2]."""
    b = scale_of(j)
    mu = f / N_MU
    out = np.empty(NSYM)
    for k in range(NSYM - 1):
        d = k - A
        lo, hi = d - 0.5 - mu, d + 0.5 - mu
        if lo >= 0.0:
            out[k] = 0.5 * (math.exp(-lo / b) - math.exp(-hi / b))
        elif hi <= 0.0:
            out[k] = 0.5 * (math.exp(hi / b) - math.exp(lo / b))
        else:
            out[k] = 1.0 - 0.5 * math.exp(lo / b) - 0.5 * math.exp(-hi / b)
    out[ESC] = 0.5 * math.exp((-A - 0.5 - mu) / b) + 0.5 * math.exp(-(A + 0.5 - mu) / b)
    return out


def freq_row(masses):
    """Integer frequencies summing to TOTAL, each at least 1."""
    fr = [1 + int(math.floor(m * (TOTAL - NSYM))) for m in masses]
    left = TOTAL - sum(fr)
    assert 0 <= left <= NSYM
    k = max(range(NSYM), key=lambda i: (fr[i], -i))
    fr[k] += left
    return fr


def freq_table():
    """[N_SCALE][N_MU][NSYM] integer frequencies."""
    return np.array([[freq_row(laplace_row_masses(j, f)) for f in range(N_MU)] for j in range(N_SCALE)],
                    dtype=np.int64)


def cum_table(freq=None):
    """[N_SCALE][N_MU][NSYM + 1] cumulative frequencies (0 .. TOTAL)."""
    freq = freq_table() if freq is None else freq
    c = np.zeros(freq.shape[:-1] + (NSYM + 1,), dtype=np.int64)
    c[..., 1:] = np.cumsum(freq, axis=-1)
    return c


# ----------------------------------------------------------------------------
# per-latent coding parameters (decided in float32)
# ----------------------------------------------------------------------------
def coding_decision(mu, s):
    """(c, f, j) of one latent from its ARM outputs, in float32 arithmetic."""
    mu32, s32 = np.float32(mu), np.float32(s)
    if np.isnan(s32):
        sc = LOG_BMAX32
    else:
        sc = min(max(s32, LOG_BMIN32), LOG_BMAX32)
    j = int(np.rint(np.float32(np.float32(sc - LOG_BMIN32) * np.float32(SCALE_PER_LN))))
    if np.isnan(mu32):
        mc = np.float32(0.0)
    else:
        mc = min(max(mu32, -MU_LIM), MU_LIM)
    fl = np.float32(np.floor(mc))
    fr = np.float32(mc - fl)
    f = int(np.rint(np.float32(fr * np.float32(N_MU))))
    c = int(fl)
    if f == N_MU:
        f, c = 0, c + 1
    return c, f, j


def escape_payload(d):
    """Raw (value, bits) symbols sent after ESC for |d| > A."""
    v = abs(d) - A
    n = v.bit_length()
    out = [(n - 1, 5)]
    r = n - 1
    first = r % 8 if r % 8 else (8 if r else 0)
    pos = r
    size = first
    while pos > 0:
        pos -= size
        out.append(((v >> pos) & ((1 << size) - 1), size))
        size = 8
    out.append((1 if d < 0 else 0, 1))
    return out


def symbols_of(d, cum_row):
    """(cum, freq) list of one latent: its primary symbol, then its escape
    payload."""
    if -A <= d <= A:
        k = d + A
        return [(int(cum_row[k]), int(cum_row[k + 1] - cum_row[k]))]
    out = [(int(cum_row[ESC]), int(cum_row[ESC + 1] - cum_row[ESC]))]
    for v, bits in escape_payload(d):
        out.append((v << (PREC - bits), 1 << (PREC - bits)))
    return out


def ideal_bits(syms):
    """-log2 of the coded probabilities of a symbol list."""
    return sum(-math.log2(fr / TOTAL) for _, fr in syms)


# ----------------------------------------------------------------------------
# decode order
# ----------------------------------------------------------------------------
def wavefront_slope(C):
    return 1 + max(dx // (-dy) for dy, dx in context_offsets(C) if dy < 0)


def level_sets(L):
    return [[0]] + ([list(range(1, L))] if L > 1 else [])


def decode_schedule(H, W, L, C):
    """For every set: (n_states, [groups]) where a group is a list of
    (state, level, i, j) in ascending state order; the groups are in decode
    order (levels of the set ascending, steps ascending, row groups
    ascending)."""
    a = wavefront_slope(C)
    shapes = level_shapes(H, W, L)
    out = []
    for levels in level_sets(L):
        n = min(MAX_LANES, shapes[levels[0]][0])
        groups = []
        for lv in levels:
            h, w = shapes[lv]
            for t in range(w + a * (h - 1)):
                i_lo = max(0, -((-(t - (w - 1))) // a))
                i_hi = min(h - 1, t // a)
                if i_lo > i_hi:
                    continue
                for g in range(i_lo // n, i_hi // n + 1):
                    rows = range(max(i_lo, g * n), min(i_hi, g * n + n - 1) + 1)
                    groups.append([(i - g * n, lv, i, t - a * i) for i in rows])
        out.append((n, groups))
    return out


# ----------------------------------------------------------------------------
# interleaved rANS
# ----------------------------------------------------------------------------
def rans_encode_rounds(n_states, rounds):
    """rounds: decode-order list of rounds, each a list of (state, cum, freq)
    in ascending state order.  Returns (final states, bytes in stream
    order)."""
    x = [RANS_L] * n_states
    emitted = []
    for rnd in reversed(rounds):
        for st, cum, fr in reversed(rnd):
            while x[st] >= ((RANS_L >> PREC) << 8) * fr:
                emitted.append(x[st] & 0xFF)
                x[st] >>= 8
        for st, cum, fr in rnd:
            x[st] = ((x[st] // fr) << PREC) + (x[st] % fr) + cum
    return x, emitted[::-1]


def _rounds_of_group(group, syms_of):
    """Rounds of one group: the primary symbols, then payload round q."""
    lists = [(st, syms_of(lv, i, j)) for st, lv, i, j in group]
    q_max = max(len(s) for _, s in lists)
    return [[(st, *s[q]) for st, s in lists if len(s) > q] for q in range(q_max)]


def coding_params(arch: Arch, H, W, yq, arm_w):
    """Per-latent (c, f, j) from the ARM outputs of the known latents
    (float64 ARM, decisions in float32), as dicts keyed by level."""
    L, C = arch.n_levels, arch.arm_ctx
    P = unpack(arch, arm_w, _ups_zeros(arch), _syn_zeros(arch))
    offs = context_offsets(C)
    out = []
    for lv, g in enumerate(split_levels(np.asarray(yq, np.float64), H, W, L)):
        mu, s, _ = arm_forward(gather_context(g, offs), P)
        out.append([coding_decision(m, ss) for m, ss in zip(mu, s)])
    return out


def _ups_zeros(arch):
    from .coolchic import param_sizes
    return np.zeros(param_sizes(arch)[1])


def _syn_zeros(arch):
    from .coolchic import param_sizes
    return np.zeros(param_sizes(arch)[2])


def _check_latents(yq):
    y = np.asarray(yq, np.float64)
    if not np.all(np.isfinite(y)) or np.any(y != np.rint(y)) or np.any(np.abs(y) > (1 << 20)):
        raise ValueError("latents must be integers of magnitude at most 2^20")


def encode(arch: Arch, H, W, yq, arm_w):
    """Bitstream (bytes) of the integer latent pyramid yq."""
    _check_latents(yq)
    L = arch.n_levels
    cum = cum_table()
    levels = split_levels(np.asarray(yq, np.float64), H, W, L)
    params = coding_params(arch, H, W, yq, arm_w)
    shapes = level_shapes(H, W, L)

    def syms_of(lv, i, j):
        c, f, sj = params[lv][i * shapes[lv][1] + j]
        return symbols_of(int(levels[lv][i, j]) - c, cum[sj, f])

    sets = []
    for n, groups in decode_schedule(H, W, L, arch.arm_ctx):
        rounds = [r for g in groups for r in _rounds_of_group(g, syms_of)]
        sets.append((n, *rans_encode_rounds(n, rounds)))
    out = bytearray(MAGIC)
    out += np.uint32(len(sets)).tobytes()
    for _, _, words in sets:
        out += np.uint32(len(words)).tobytes()
    for _, x, _ in sets:
        out += np.asarray(x, np.uint32).tobytes()
    for _, _, words in sets:
        out += bytes(words)
    return bytes(out)


def _find_symbol(cum_row, slot):
    k = 0
    while not (cum_row[k] <= slot < cum_row[k + 1]):
        k += 1
    return k


def decode(arch: Arch, H, W, data, arm_w):
    """Latent pyramid (float64, integer values) from a bitstream: every latent
    in the wavefront order, its ARM evaluated on the already decoded
    context (float64, decisions in float32)."""
    L, C = arch.n_levels, arch.arm_ctx
    cum = cum_table()
    P = unpack(arch, arm_w, _ups_zeros(arch), _syn_zeros(arch))
    offs = context_offsets(C)
    shapes = level_shapes(H, W, L)
    grids = [np.zeros(s) for s in shapes]
    if data[:4] != MAGIC:
        raise ValueError("not a latent bitstream")
    sched = decode_schedule(H, W, L, C)
    n_sets = int(np.frombuffer(data, np.uint32, 1, 4)[0])
    if n_sets != len(sched):
        raise ValueError("set count does not match the problem")
    o = 8
    n_words = np.frombuffer(data, np.uint32, n_sets, o).astype(np.int64); o += 4 * n_sets
    states = []
    for n, _ in sched:
        states.append([int(v) for v in np.frombuffer(data, np.uint32, n, o)]); o += 4 * n
    streams = []
    for nw in n_words:
        streams.append(list(data[o:o + int(nw)])); o += int(nw)
    if o != len(data):
        raise ValueError("bitstream length does not match its header")

    def context(lv, i, j):
        g = grids[lv]
        h, w = shapes[lv]
        return np.array([[g[i + dy, j + dx] if 0 <= i + dy < h and 0 <= j + dx < w else 0.0 for dy, dx in offs]])

    for (n, groups), x, words in zip(sched, states, streams):
        pos = 0

        def round_(items):
            nonlocal pos
            out = {}
            for st, cum_row in items:
                slot = x[st] & (TOTAL - 1)
                k = _find_symbol(cum_row, slot)
                x[st] = int(cum_row[k + 1] - cum_row[k]) * (x[st] >> PREC) + slot - int(cum_row[k])
                out[st] = k
            for st, _ in items:
                while x[st] < RANS_L:
                    x[st] = (x[st] << 8) | words[pos]
                    pos += 1
            return out

        def raw_row(bits):
            return np.arange(0, TOTAL + 1, 1 << (PREC - bits))

        for group in groups:
            info = {}
            for st, lv, i, j in group:
                mu, s, _ = arm_forward(context(lv, i, j), P)
                c, f, sj = coding_decision(mu[0], s[0])
                info[st] = (lv, i, j, c, cum[sj, f])
            prim = round_([(st, info[st][4]) for st, *_ in group])
            esc = [st for st in prim if prim[st] == ESC]
            vals = {st: prim[st] - A for st in prim if prim[st] != ESC}
            if esc:
                # payload round 1: the bit length; then round q holds the
                # (q-1)-th remaining symbol of every escaped latent (bit
                # chunks, most significant first, then the sign)
                nbits = round_([(st, raw_row(5)) for st in esc])
                plan = {}
                for st in esc:
                    r = nbits[st]
                    sizes = ([r % 8 or 8] + [8] * ((r - (r % 8 or 8)) // 8)) if r else []
                    plan[st] = sizes + [1]
                v = {st: 1 for st in esc}
                neg = {}
                q = 0
                while any(len(plan[st]) > q for st in esc):
                    act = [st for st in esc if len(plan[st]) > q]
                    got = round_([(st, raw_row(plan[st][q])) for st in act])
                    for st in act:
                        if q == len(plan[st]) - 1:
                            neg[st] = got[st]
                        else:
                            v[st] = (v[st] << plan[st][q]) | got[st]
                    q += 1
                for st in esc:
                    mag = v[st] + A
                    vals[st] = -mag if neg[st] else mag
            for st, (lv, i, j, c, _) in info.items():
                grids[lv][i, j] = c + vals[st]
        if pos != len(words) or any(v != RANS_L for v in x):
            raise ValueError("bitstream inconsistent with the problem")
    return np.concatenate([g.ravel() for g in grids])
