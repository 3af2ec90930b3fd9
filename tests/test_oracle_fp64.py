"""Pins of the oracle's fp64 statement of the method (the reference for the
reported |D_gpu - D_fp64|): its branch and bound equals the dense definition
on its own grid (d_j = d_lo + (d_hi - d_lo) j 2^-L in fp64, keys from the fp64
point value), and it agrees with the fp32 statement to within a few grid
steps on the 128x128 config."""

import numpy as np
import pytest

from synth import config_windows


@pytest.mark.parametrize("k", range(6))
def test_bnb64_equals_its_dense_definition_tiny(orc, k):
    w = config_windows("tiny", [k])[0]
    s = w.spec
    ev = orc.Events.of_window(w)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    span = float(s.d_hi) - float(s.d_lo)
    best = None
    for j in range(1, 1 << L):
        d = float(s.d_lo) + span * np.ldexp(float(j), -L)
        S, N = orc.point64(ev, d)
        K = orc.key(ev.M, S, N)
        if best is None or K > best[0]:
            best = (K, j, d)
    r, d64 = orc.bnb64(ev, s.d_lo, s.d_hi, s.eps)
    assert (r.K, r.j_star) == best[:2]
    assert d64 == best[2]


@pytest.mark.parametrize("k", range(3))
def test_bnb64_agrees_with_fp32_statement(orc, k):
    w = config_windows("c1", [k])[0]
    s = w.spec
    ev = orc.Events.of_window(w)
    r32 = orc.bnb(ev, s.d_lo, s.d_hi, s.eps)
    r64, d64 = orc.bnb64(ev, s.d_lo, s.d_hi, s.eps)
    assert r64.status == 0 and r32.status == 0
    assert abs(r32.d_hat - d64) <= 4 * s.eps
    assert abs(d64 - s.d_true) < 0.02
