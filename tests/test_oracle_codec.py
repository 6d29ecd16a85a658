"""Pins of the oracle's entropy coder (oracle/codec.py) against things other
than itself: scipy's Laplace distribution for the table masses, hand-worked
decisions and escape payloads, the closed form of one rANS step, the
information identity of rANS (bytes written plus the final states' content
equal the coded symbols' information up to the coder's precision loss),
brute-force round trips, a brute-force causality check of the decode order,
and the training rate of Eq. (1) for the measured size of the bitstream."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as O
import oracle.codec as K
from paper_2403_11651_amd import workloads as WL


@pytest.fixture(scope="module")
def freq():
    return K.freq_table()


def test_table_masses_match_scipy_laplace():
    for j in (0, 1, 17, 40, 63, 74):
        b = math.exp(float(np.float32(math.log(0.01))) + j / 8)
        for f in (0, 3, 8, 15):
            mu = f / 16
            d = np.arange(-48, 49)
            ref = scipy.stats.laplace.cdf(d + 0.5, mu, b) - scipy.stats.laplace.cdf(d - 0.5, mu, b)
            esc = scipy.stats.laplace.cdf(-48.5, mu, b) + scipy.stats.laplace.sf(48.5, mu, b)
            got = K.laplace_row_masses(j, f)
            assert np.allclose(got[:-1], ref, rtol=1e-12, atol=1e-15), (j, f)
            assert math.isclose(got[-1], esc, rel_tol=1e-12, abs_tol=1e-300), (j, f)


def test_frequencies_from_scipy_masses(freq):
    """Every row: frequency = 1 + floor(mass (2^16 - 98)) from scipy's
    masses, the remainder on the first most frequent symbol, total 2^16."""
    assert freq.shape == (75, 16, 98)
    assert np.all(freq.sum(-1) == 65536) and freq.min() >= 1
    for j in (0, 5, 30, 52, 74):
        b = math.exp(float(np.float32(math.log(0.01))) + j / 8)
        for f in (0, 7, 8, 12):
            mu = f / 16
            d = np.arange(-48, 49)
            m = np.append(scipy.stats.laplace.cdf(d + 0.5, mu, b) - scipy.stats.laplace.cdf(d - 0.5, mu, b),
                          scipy.stats.laplace.cdf(-48.5, mu, b) + scipy.stats.laplace.sf(48.5, mu, b))
            base = 1 + np.floor(m * (65536 - 98)).astype(np.int64)
            top = int(np.argmax(base))
            diff = freq[j, f] - base
            assert np.all(np.delete(diff, top) == 0), (j, f)
            assert diff[top] == 65536 - base.sum()


def test_table_symmetries_and_extremes(freq):
    # mean 0: symmetric about d = 0; mean 1/2: mirror d <-> 1 - d, except the
    # tie at the centre, whose remainder goes to d = 0 (the first)
    for j in range(75):
        r = freq[j, 0, :97]
        assert np.array_equal(r, r[::-1]), j
        h = freq[j, 8, :97]
        assert np.array_equal(h[50:], h[1:48][::-1]) and h[48] >= h[49], j
    # b = 0.01: all the mass at d = 0 (floors elsewhere); b ~ 100: the escape
    # takes about exp(-48.5 / b) of the total
    assert freq[0, 0, 48] == 65536 - 97 and np.all(np.delete(freq[0, 0], 48) == 1)
    b = math.exp(float(np.float32(math.log(0.01))) + 74 / 8)
    assert abs(freq[74, 0, 97] / 65536 - math.exp(-48.5 / b)) < 2e-3


@pytest.mark.parametrize("mu,s,expect", [
    (2.03, 0.0, (2, 0, 37)),            # frac 0.03 -> rint(0.48) = 0
    (-0.97, 0.0, (-1, 0, 37)),          # floor -1, frac 0.03
    (0.97, 0.0, (1, 0, 37)),            # rint(15.52) = 16 carries into c
    (1.0 / 32, 0.0, (0, 0, 37)),        # 16 frac = 0.5: tie to even
    (3.0 / 32, 0.0, (0, 2, 37)),        # 1.5 -> 2
    (5.5, math.log(0.01), (5, 8, 0)),
    (-3.25, math.log(100.0), (-4, 12, 74)),
    (0.0, -50.0, (0, 0, 0)),
    (0.0, 50.0, (0, 0, 74)),
    (float("nan"), float("nan"), (0, 0, 74)),
    (3e7, 0.0, (1 << 20, 0, 37)),
])
def test_coding_decision_hand_values(mu, s, expect):
    # s = 0: 8 (0 - ln 0.01) = 36.84 -> 37
    assert K.coding_decision(mu, s) == expect


def test_scale_index_tie():
    s = np.float32(np.float32(math.log(0.01)) + np.float32(1.0 / 16))
    # the float32 difference is exactly 1/16 here, so 8 * (s - ln 0.01) = 1/2
    assert np.float32(s - np.float32(math.log(0.01))) == np.float32(1.0 / 16)
    assert K.coding_decision(0.0, s)[2] == 0


def test_escape_payload_hand_values():
    assert K.escape_payload(49) == [(0, 5), (0, 1)]
    assert K.escape_payload(-49) == [(0, 5), (1, 1)]
    # |d| - 48 = 300 = 0b1_0010_1100: 9 bits, 8 below the leading one
    assert K.escape_payload(348) == [(8, 5), (0b00101100, 8), (0, 1)]
    # |d| - 48 = 2097104 = 0b1_1111_1111_1111_1101_0000: 21 bits, 20 below it
    assert K.escape_payload(-(2 ** 21)) == [(20, 5), (0b1111, 4), (0xFF, 8), (0xD0, 8), (1, 1)]


def test_one_rans_step_closed_form():
    # one 1-bit symbol (cum 2^15, freq 2^15) from the initial state 2^23:
    # x' = floor(2^23 / 2^15) 2^16 + 2^23 mod 2^15 + 2^15 = 2^24 + 2^15
    x, out = K.rans_encode_rounds(1, [[(0, 1 << 15, 1 << 15)]])
    assert x == [(1 << 24) + (1 << 15)] and out == []


def _random_rounds(rng, n_states, n_rounds):
    rounds = []
    for _ in range(n_rounds):
        rnd = []
        for st in range(n_states):
            if rng.random() < 0.8:
                fr = int(rng.choice([1, 2, 7, 300, 4096, 40000, 65000]))
                rnd.append((st, int(rng.integers(0, 65536 - fr + 1)), fr))
        rounds.append(rnd)
    return rounds


def test_rans_information_identity():
    """8 x bytes written + sum over states of log2(x_final / 2^23) equals the
    information of the coded symbols up to the coder's rounding, which the
    state's 7 bits of headroom bound by -log2(1 - 2^-7) per symbol."""
    rng = np.random.default_rng(5)
    for n_states in (1, 3, 64):
        rounds = _random_rounds(rng, n_states, 300)
        x, out = K.rans_encode_rounds(n_states, rounds)
        info = sum(-math.log2(fr / 65536) for rnd in rounds for _, _, fr in rnd)
        n_sym = sum(len(r) for r in rounds)
        measured = 8 * len(out) + sum(math.log2(v / (1 << 23)) for v in x)
        assert all((1 << 23) <= v < (1 << 31) for v in x)
        # each step maps x to within a factor (1 -+ 2^-7) of x 2^16 / freq
        assert abs(measured - info) <= n_sym * -math.log2(1 - 2 ** -7), (n_states, measured, info)


def _small_problem(seed, arch, H, W, big=()):
    rng = np.random.default_rng(seed)
    n = sum((H >> l) * (W >> l) for l in range(arch.n_levels))
    y = np.rint(rng.laplace(0, 2, n))
    for k, v in big:
        y[k] = v
    na, _, _ = O.param_sizes(arch)
    return y, rng.normal(0, 0.1, na)


@pytest.mark.parametrize("arch,H,W", [(O.Arch(3, 8, 2, 8, 16, 1), 16, 24), (O.Arch(4, 24, 2, 8, 16, 1), 32, 40),
                                      (O.Arch(2, 16, 1, 8, 16, 1), 40, 24), (O.Arch(1, 8, 3, 8, 16, 1), 8, 72)])
def test_round_trip_with_escapes(arch, H, W):
    y, w = _small_problem(7, arch, H, W, big=((5, 300), (7, -1000), (11, -49), (12, 49), (3, 2 ** 20)))
    data = K.encode(arch, H, W, y, w)
    assert np.array_equal(K.decode(arch, H, W, data, w), y)
    bad = bytearray(data)
    bad[-1] ^= 0x5A
    with pytest.raises(Exception):
        assert not np.array_equal(K.decode(arch, H, W, bytes(bad), w), y)
        raise ValueError("corrupt stream decoded to the same latents")


def test_rejects_non_integer_or_huge_latents():
    arch = O.Arch(2, 8, 1, 8, 16, 1)
    y, w = _small_problem(1, arch, 8, 8)
    y2 = y.copy(); y2[0] = 0.5
    with pytest.raises(ValueError):
        K.encode(arch, 8, 8, y2, w)
    y2[0] = 2 ** 20 + 1
    with pytest.raises(ValueError):
        K.encode(arch, 8, 8, y2, w)


@pytest.mark.parametrize("C", [8, 16, 24])
def test_decode_order_is_causal_and_complete(C):
    """Brute force: every latent is decoded once, and each of its causal
    neighbours inside the grid is decoded in an earlier step of the same
    grid."""
    H, W, L = 24, 40, 3
    offs = O.context_offsets(C)
    for n, groups in K.decode_schedule(H, W, L, C):
        when = {}
        step = -1
        last = None
        for g in groups:
            lv, i, j = g[0][1], g[0][2], g[0][3]
            key = (lv, K.wavefront_slope(C) * i + j)
            if key != last:
                step += 1
                last = key
            for st, lv2, i2, j2 in g:
                assert st == i2 % n and (lv2, i2, j2) not in when
                when[(lv2, i2, j2)] = step
        for (lv, i, j), t in when.items():
            h, w = H >> lv, W >> lv
            for dy, dx in offs:
                if 0 <= i + dy < h and 0 <= j + dx < w:
                    assert when[(lv, i + dy, j + dx)] < t, (lv, i, j, dy, dx)
        levels = {lv for lv, _, _ in when}
        assert len(when) == sum((H >> lv) * (W >> lv) for lv in levels)


def _rate_case(arm_std, unit_latents=False):
    arch = O.TINY
    H = W = 64
    na, nu, ns = O.param_sizes(arch)
    if unit_latents:
        n = sum((H >> l) * (W >> l) for l in range(arch.n_levels))
        y = np.rint(np.random.default_rng(1).laplace(0.0, 1.0, n))
    else:
        y = np.rint(WL.latents(1, H, W, arch.n_levels))
    w = WL.weights(2, na + nu + ns)
    arm = w[:na] * (arm_std / 0.1)
    img = WL.image(0, H, W, 12)
    data = K.encode(arch, H, W, y, arm)
    fwd = O.forward(arch, img, y, arm, w[na:na + nu], w[na + nu:], 1e-3)
    # payload information: the coded bytes, plus log2(x / 2^23) bits held by
    # each final state (64 states for level 0, 32 for levels 1-6)
    n_states = 64 + 32
    x = np.frombuffer(data, np.uint32, n_states, 16).astype(np.float64)
    header = 16 + 4 * n_states
    return 8 * (len(data) - header) + np.log2(x / 2.0 ** 23).sum(), fwd["R"], fwd["rate"]


def test_bitstream_size_tracks_the_training_rate():
    """Latents drawn from Laplace(0, 1) and ARM weights of N(0, 0.01^2), so
    every predicted scale is near 1 and no latent is near the probability
    floor: the information a 64x64 pyramid's bitstream carries (its coded
    bytes and the content of the final coder states) is within 1 % of the
    rate term of Eq. (1) for the same latents and ARM (the difference: the
    quantised Laplace parameters, the floor and the coder)."""
    bits, R, rate = _rate_case(0.01, unit_latents=True)
    assert rate.max() < 16.0
    assert abs(bits - R) <= 0.01 * R, (bits, R)


def test_probability_floor_caps_extreme_latents():
    """With N(0, 0.1^2) ARM weights some predicted scales are far too small
    and a latent can cost over 30 bits under the Laplace model; the floor
    (frequency >= 1 of 2^16) caps a symbol without escape at 16 bits, so the
    bitstream carries less than R and at most about sum(min(r, 16))."""
    bits, R, rate = _rate_case(0.1)
    assert rate.max() > 30.0
    capped = np.minimum(rate, 16.0).sum()
    assert bits <= 1.01 * capped, (bits, capped, R)
    assert bits < R
