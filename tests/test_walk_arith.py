"""Arithmetic facts the evaluation kernel's walk relies on for bit-exact
corner decisions (eq. (17)): the fp64 difference between a pixel edge and an
event coordinate is exact, so computing it from an origin moved by the step
direction gives the very same value, and so the very same decision, as the
direct form.  Pure host arithmetic, no GPU."""

import numpy as np


def test_shifted_origin_difference_is_exact():
    rng = np.random.default_rng(7)
    n = 1_000_000
    # event coordinates: fp32 values over the sensor range, including tiny and negative ones
    x = np.concatenate([rng.uniform(-2.0, 2000.0, n).astype(np.float32),
                        (rng.standard_normal(n // 10) * 1e-3).astype(np.float32)])
    k = rng.integers(-1, 2001, x.size)
    for p in (0, 1):
        direct = (k + p).astype(np.float64) - x.astype(np.float64)
        shifted = k.astype(np.float64) - (x.astype(np.float64) - p)
        assert np.array_equal(direct, shifted)
        # and both are the exact difference (checked in integer units of 2^-149)
        exact = [(int(kk) + p) * 2**149 - int(np.float64(xx) * 2**149) for kk, xx in zip(k[:2000], x[:2000])]
        assert [int(v * 2**149) for v in direct[:2000]] == exact
