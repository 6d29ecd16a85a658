"""Pins of the oracle's Philox4x32-10 noise generator."""
import numpy as np

from oracle import noise as N


def test_philox_known_answers():
    """Known-answer vectors published with the Random123 library for
    Philox4x32 with 10 rounds."""
    assert N.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    f = 0xFFFFFFFF
    assert N.philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert N.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_noise_range_and_moments():
    u = N.uniform_noise(40000, seed=123, it=5, stream_id=2)
    assert u.min() >= -0.5 and u.max() < 0.5
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 12.0) < 0.002
    # values are multiples of 2^-24 (exact in float32)
    assert np.all(((u.astype(np.float64) + 0.5) * 2 ** 24) % 1 == 0)


def test_noise_depends_on_every_counter_word():
    a = N.uniform_noise(64, seed=1)
    for kw in (dict(seed=2), dict(seed=1, it=1), dict(seed=1, stream_id=1), dict(seed=1 << 32)):
        b = N.uniform_noise(64, **kw)
        assert not np.array_equal(a, b), kw
    assert np.array_equal(a[:32], N.uniform_noise(32, seed=1))
