"""The endpoint certificate of an interval's bound, pinned on the CPU.

For an interval [d_a, d_b] the library may first compute, from the endpoint
pixels alone, U = sum over the events inside the image at both ends of
|dkx| + |dky| + 1 and claims K_bar >= U^2 - N_low^2 (eqs. (15)-(20)): such an
event's staircase walk visits at least that many distinct image pixels, so
U <= sum of the bound image, and Cauchy-Schwarz over the M cells gives
M * S_bar >= (sum H_bar)^2.  With the point values (S_e, N_e) at an end d_e
of the interval it also claims K_bar >= M S_e + max(0, U - N_e)^2 - N_low^2:
H_bar >= H(d_e) pixel by pixel, so S_bar >= S_e + (sum (H_bar - H(d_e)))^2 / M.
These tests take the endpoint pixels from the independent NumPy warp and the
bound and point images from the oracle, and check every link of both chains,
on every depth of the grid and on single events.
"""

import numpy as np
import pytest

from synth import config_windows
from tests import npwarp


def _endpoints(ev, d_a, d_b):
    pa = npwarp.pixels(ev.x, ev.y, ev.t, ev.tau, ev.W, ev.H, ev.cx, ev.cy, d_a)
    pb = npwarp.pixels(ev.x, ev.y, ev.t, ev.tau, ev.W, ev.H, ev.cx, ev.cy, d_b)
    full = (pa >= 0) & (pb >= 0)
    walk = np.abs(pb % ev.W - pa % ev.W) + np.abs(pb // ev.W - pa // ev.W) + 1
    return full, walk


def _windows():
    ws = [config_windows("c1", [0])[0], config_windows("c2", [2], n_events=8000)[0]]
    ws += config_windows("tiny", range(3))
    return ws


@pytest.mark.parametrize("k", range(5))
def test_certificate_is_below_the_bound(orc, k):
    w = _windows()[k]
    ev = orc.Events.of_window(w)
    s = w.spec
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    rng = np.random.default_rng(30 + k)
    for depth in range(1, min(L, 9) + 1):
        step = 1 << (L - depth)
        for j in rng.choice(1 << depth, size=min(4, 1 << depth), replace=False):
            d_a = orc.grid_d(s.d_lo, s.d_hi, L, int(j) * step)
            d_b = orc.grid_d(s.d_lo, s.d_hi, L, (int(j) + 1) * step)
            S, N, img = orc.bound(ev, d_a, d_b, want_image=True)
            full, walk = _endpoints(ev, d_a, d_b)
            U = int(walk[full].sum())
            assert N == int(full.sum())  # N_low: both endpoints inside (eq. (20))
            assert U <= int(img.sum(dtype=np.int64))  # each such walk visits |dkx| + |dky| + 1 image pixels
            assert ev.M * S >= int(img.sum(dtype=np.int64)) ** 2  # Cauchy-Schwarz
            Kb = orc.key(ev.M, S, N)
            assert Kb >= U * U - N * N, (depth, j)
            # either end d_e of the interval: H_bar >= H(d_e) pixel by pixel
            for d_e in (d_a, d_b):
                Se, Ne, He = orc.point(ev, d_e, want_image=True)
                assert np.all(img >= He)
                X = max(0, U - Ne)  # sum(H_bar - H(d_e)) >= U - N_e
                assert ev.M * S >= ev.M * Se + X * X
                assert Kb >= ev.M * Se + X * X - N * N, (depth, j, d_e)


def test_single_event_walk_visits_at_least_its_manhattan_length(orc):
    """One event at a time: the bound image of a full event has at least
    |dkx| + |dky| + 1 non-zero pixels (exactly that many plus one per
    two-sided corner), all in the image."""
    base = config_windows("c1", [1])[0]
    s = base.spec
    rng = np.random.default_rng(5)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    checked = 0
    for i in rng.choice(base.x.size, size=60, replace=False):
        ev = orc.Events(base.x[i:i + 1], base.y[i:i + 1], base.t_rel[i:i + 1], s.tau, s.width, s.height, s.foe)
        for depth in (1, 3, 6):
            step = 1 << (L - depth)
            j = int(rng.integers(0, 1 << depth))
            d_a = orc.grid_d(s.d_lo, s.d_hi, L, j * step)
            d_b = orc.grid_d(s.d_lo, s.d_hi, L, (j + 1) * step)
            _, N, img = orc.bound(ev, d_a, d_b, want_image=True)
            full, walk = _endpoints(ev, d_a, d_b)
            if full[0]:
                assert N == 1 and int(np.count_nonzero(img)) >= int(walk[0])
                assert int(img.max()) == 1  # a walk never visits a pixel twice
                checked += 1
    assert checked > 50
