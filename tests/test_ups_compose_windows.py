"""Host-side pin of the fact the composed coarse upsampling adjoint of the
HIP path relies on (Section II upsampling, Table I "TConv"): after m steps of
the clamped stride-2 transposed convolution, column q of the 1-D product of
the steps (the image of the unit vector at coarse index q) is zero outside
rows [2^m q - 3 (2^m - 1), 2^m q + 4 (2^m - 1)], borders included.  Checked
with the oracle's own 1-D transposed convolution and random taps."""
import numpy as np
import pytest

import oracle.coolchic as O


@pytest.mark.parametrize("n,m", [(2, 1), (3, 2), (8, 3), (5, 4), (12, 4), (1, 3)])
def test_composed_columns_stay_in_their_windows(n, m):
    rng = np.random.default_rng(100 * n + m)
    taps = rng.normal(size=(m, 8)) + 0.1  # no zero taps: every reachable row is nonzero
    for q in range(n):
        col = np.zeros(n)
        col[q] = 1.0
        for k in range(m):
            col = O.tconv1d(col, taps[k], axis=-1)
        lo, hi = (1 << m) * q - 3 * ((1 << m) - 1), (1 << m) * q + 4 * ((1 << m) - 1)
        rows = np.nonzero(col)[0]
        assert col.size == n << m
        assert rows.min() >= max(lo, 0) and rows.max() <= min(hi, col.size - 1), (n, m, q, rows.min(), rows.max())
        # the window is tight away from the borders
        if lo >= 0 and hi < col.size:
            assert rows.min() == lo and rows.max() == hi
