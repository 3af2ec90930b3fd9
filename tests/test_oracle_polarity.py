"""Pins of the oracle's polarity-aware contrast (the event image of eq. (13)
kept per polarity, contrast over both images together: K = 2M S - N^2).

Checked against an independent NumPy statement (the warp of tests/npwarp.py
and np.bincount over 2M cells), a closed form (a window doubled with
opposite polarities has four times the polarity-blind key at every d and
every interval, so Algorithm 1 takes the same decisions), the
bound's validity, a brute-force sweep on tiny windows, and symmetries.
"""

import numpy as np
import pytest

from synth import config_windows
from tests import npwarp

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _np_pol_image(w, d):
    s = w.spec
    M = s.width * s.height
    pix = npwarp.pixels(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe[0], s.foe[1], d)
    keep = pix >= 0
    cell = pix[keep] + M * (w.p[keep] > 0)
    return np.bincount(cell, minlength=2 * M).astype(np.int64)


def _key(M2, H):
    S = int((H.astype(object) ** 2).sum())
    N = int(H.sum())
    return M2 * S - N * N, S, N


@pytest.mark.parametrize("cfg,n", [("c1", None), ("c2", 20_000)])
def test_point_pol_is_bincount_over_two_images(orc, cfg, n):
    kw = {"n_events": n} if n else {}
    w = config_windows(cfg, [2], **kw)[0]
    s = w.spec
    ev = orc.Events.of_window(w, polarity=True)
    assert (w.p > 0).any() and (w.p <= 0).any()
    for d in [0.0, float(np.float32(s.d_true)), float(np.float32(0.37 * s.d_hi))]:
        H = _np_pol_image(w, d)
        S, N, img = orc.point_pol(ev, d, want_image=True)
        assert np.array_equal(img.astype(np.int64), H), d
        _, S0, N0 = _key(2 * ev.M, H)
        assert (S, N) == (S0, N0)


def _doubled(w):
    """The window's events twice: once all positive, once all negative."""
    from oracle import oracle as O

    s = w.spec
    x = np.concatenate([w.x, w.x])
    y = np.concatenate([w.y, w.y])
    t = np.concatenate([w.t_rel, w.t_rel])
    p = np.concatenate([np.ones(w.n, np.int8), -np.ones(w.n, np.int8)])
    return O.Events(x, y, t, s.tau, s.width, s.height, s.foe, p)


def test_doubled_window_closed_form(orc):
    """Both images equal the blind image H: S' = 2S, N' = 2N, so
    K' = 2M(2S) - (2N)^2 = 4K at every d, and the canonical optimum agrees."""
    w = config_windows("c1", [3])[0]
    s = w.spec
    ev = orc.Events.of_window(w)
    ev2 = _doubled(w)
    for d in [0.0, 0.2, float(np.float32(s.d_true))]:
        S, N = orc.point(ev, d)
        S2, N2 = orc.point_pol(ev2, d)
        assert (S2, N2) == (2 * S, 2 * N)
        assert orc.key(2 * ev.M, S2, N2) == 4 * orc.key(ev.M, S, N)
        Sb, Nb = orc.bound(ev, 0.05, d + 0.1)
        Sb2, Nb2 = orc.bound_pol(ev2, 0.05, d + 0.1)
        assert (Sb2, Nb2) == (2 * Sb, 2 * Nb)
    r = orc.bnb(ev, s.d_lo, s.d_hi, s.eps)
    r2 = orc.bnb_pol(ev2, s.d_lo, s.d_hi, s.eps)
    assert (r2.j_star, r2.K) == (r.j_star, 4 * r.K)
    # every key, bounds included, is scaled by 4: Algorithm 1 takes the same
    # decisions, node for node
    trace = lambda q: (q.nodes_expanded, q.nodes_pruned, q.point_evals, q.bound_evals)  # noqa: E731
    assert trace(r2) == trace(r)


def test_bound_pol_dominates_points(orc):
    """Eqs. (15)-(20) per image: every cell of the bound images is at least
    the point images' count for any fp32 d in the interval, and the bound
    key is at least every point key there."""
    w = config_windows("c2", [4], n_events=20_000)[0]
    s = w.spec
    ev = orc.Events.of_window(w, polarity=True)
    rng = np.random.default_rng(5)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    for _ in range(6):
        ja = int(rng.integers(0, (1 << L) - 64))
        jb = ja + int(rng.choice([2, 64, 4096]))
        jb = min(jb, 1 << L)
        da, db = orc.grid_d(s.d_lo, s.d_hi, L, ja), orc.grid_d(s.d_lo, s.d_hi, L, jb)
        Sb, Nb, Hb = orc.bound_pol(ev, da, db, want_image=True)
        Kb = orc.key(2 * ev.M, Sb, Nb)
        for d in np.linspace(da, db, 5).astype(np.float32):
            S, N, H = orc.point_pol(ev, float(d), want_image=True)
            assert (Hb >= H).all()
            assert Kb >= orc.key(2 * ev.M, S, N)


@pytest.mark.parametrize("k", range(8))
def test_bnb_pol_equals_brute_force_tiny(orc, k):
    """The canonical optimum (largest K, then smallest j) over the whole grid,
    computed with NumPy from the independent warp, is what Algorithm 1 returns."""
    w = config_windows("tiny", [k])[0]
    s = w.spec
    ev = orc.Events.of_window(w, polarity=True)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    best = None
    for j in range(1, 1 << L):
        d = orc.grid_d(s.d_lo, s.d_hi, L, j)
        K, _, _ = _key(2 * ev.M, _np_pol_image(w, d))
        if best is None or K > best[0]:
            best = (K, j)
    r = orc.bnb_pol(ev, s.d_lo, s.d_hi, s.eps)
    assert r.status == 0 and (r.K, r.j_star) == best


def test_polarity_flip_and_single_polarity(orc):
    w = config_windows("c1", [5])[0]
    s = w.spec
    ev = orc.Events.of_window(w, polarity=True)
    flip = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe, -w.p)
    a, b = orc.bnb_pol(ev, s.d_lo, s.d_hi, s.eps), orc.bnb_pol(flip, s.d_lo, s.d_hi, s.eps)
    assert (a.j_star, a.K) == (b.j_star, b.K)
    # the 1/0 encoding (0 = OFF) is the same split as +1/-1
    zero = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe, (w.p > 0).astype(np.int8))
    for d in [0.1, 0.3]:
        assert orc.point_pol(zero, d) == orc.point_pol(ev, d)
        assert orc.bound_pol(zero, 0.05, d) == orc.bound_pol(ev, 0.05, d)
    one = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe, np.ones(w.n, np.int8))
    blind = orc.Events.of_window(w)
    for d in [0.1, 0.3]:
        assert orc.point_pol(one, d) == orc.point(blind, d)
        assert orc.bound_pol(one, 0.05, d) == orc.bound(blind, 0.05, d)
