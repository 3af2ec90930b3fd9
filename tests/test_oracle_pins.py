"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
independent NumPy statement of the warp, library routines (bincount, var),
closed forms, invariants proved in the paper, brute force over the continuum
on tiny inputs, and recovery of the generator's true divergence.
"""

import numpy as np
import pytest

from synth import config_windows
from tests import npwarp

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _ev(orc, w, **kw):
    return orc.Events.of_window(w)


def _f32_between(lo, hi, n, rng):
    """n random fp32 values in [lo, hi] (uniform over the fp32 encodings;
    valid for 0 <= lo <= hi)."""
    a = np.array([lo], np.float32).view(np.uint32)[0]
    b = np.array([hi], np.float32).view(np.uint32)[0]
    bits = rng.integers(int(a), int(b) + 1, n, dtype=np.int64).astype(np.uint32)
    return bits.view(np.float32)


# ---------------------------------------------------------------- P1 pixels

@pytest.mark.parametrize("cfg,n", [("c1", None), ("c2", 20_000)])
def test_pixels_match_independent_numpy_warp(orc, cfg, n):
    """Eq. (12)-(13): pixel index of every event equals an independent
    NumPy fp32 statement (non-square c2 sensor catches an x/y swap)."""
    kw = {"n_events": n} if n else {}
    w = config_windows(cfg, [0], **kw)[0]
    ev = _ev(orc, w)
    rng = np.random.default_rng(1)
    s = w.spec
    ds = list(_f32_between(s.d_lo, s.d_hi * 0.999, 12, rng)) + [0.0, s.d_true]
    for d in ds:
        d = float(np.float32(d))
        got = orc.pixels(ev, d)
        ref = npwarp.pixels(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe[0], s.foe[1], d)
        assert np.array_equal(got.astype(np.int64), ref), d


# ---------------------------------------------------------------- P2 contrast

@pytest.mark.parametrize("cfg,n", [("c1", None), ("c2", 30_000)])
def test_point_value_is_bincount_and_variance(orc, cfg, n):
    """Eqs. (13)-(14) and the variance rewrite: S = sum H^2, N = sum H of
    np.bincount, and K/M^2 equals the population variance np.var(H)."""
    kw = {"n_events": n} if n else {}
    w = config_windows(cfg, [1], **kw)[0]
    ev = _ev(orc, w)
    s = w.spec
    M = s.width * s.height
    for d in (0.0, 0.1, float(np.float32(s.d_true)), 0.77):
        pix = npwarp.pixels(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe[0], s.foe[1], d)
        Hh = np.bincount(pix[pix >= 0], minlength=M).astype(np.int64)
        S, N, img = orc.point(ev, d, want_image=True)
        assert np.array_equal(img.astype(np.int64), Hh)
        assert S == int((Hh * Hh).sum()) and N == int(Hh.sum())
        K = orc.key(M, S, N)
        assert K >= 0
        assert K / M / M == pytest.approx(float(np.var(Hh.astype(np.float64))), rel=1e-12, abs=1e-15)


def test_key_closed_forms(orc):
    """All events in one pixel: K = (M - 1) N^2.  One event per pixel over the
    whole sensor: the image is flat and K = 0."""
    W, H = 9, 7
    M = W * H
    n = 13
    x = np.full(n, 3.25, np.float32)
    y = np.full(n, 5.5, np.float32)
    t = np.full(n, 0.5, np.float32)  # t' = tau: the event never moves
    ev = orc.Events(x, y, t, 0.5, W, H, (4.5, 3.5))
    S, N = orc.point(ev, 0.37)
    assert (S, N) == (n * n, n)
    assert orc.key(M, S, N) == (M - 1) * n * n
    gx, gy = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    ev2 = orc.Events(gx.ravel(), gy.ravel(), np.zeros(M, np.float32), 0.5, W, H, (4.5, 3.5))
    S, N = orc.point(ev2, 0.0)
    assert (S, N) == (M, M) and orc.key(M, S, N) == 0


# ---------------------------------------------------------------- P4 warp

def test_warp_identities(orc):
    """Eq. (12): d = 0 leaves every event in place; so do t' = tau and an
    event at the FOE, for any d."""
    w = config_windows("c1", [2])[0]
    ev = _ev(orc, w)
    s = w.spec
    base = np.floor(w.y).astype(np.int64) * s.width + np.floor(w.x).astype(np.int64)
    assert np.array_equal(orc.pixels(ev, 0.0).astype(np.int64), base)
    tt = np.full(w.n, np.float32(s.tau), np.float32)
    ev_t = orc.Events(w.x, w.y, tt, s.tau, s.width, s.height, s.foe)
    assert np.array_equal(orc.pixels(ev_t, 0.9).astype(np.int64), base)
    x = np.full(5, 64.0, np.float32)
    y = np.full(5, 64.0, np.float32)
    ev_c = orc.Events(x, y, np.zeros(5, np.float32), s.tau, s.width, s.height, s.foe)
    assert np.all(orc.pixels(ev_c, 0.95) == 64 * 128 + 64)


def test_signal_events_collapse_at_true_divergence(orc):
    """Eqs. (5)-(12): without noise, every event of one surface point warps
    to the point's end position at d = D, so they share a pixel; at a wrong d
    they spread.  A wrong sign or a swapped t/tau fails this."""
    w = config_windows("noisefree", [0])[0]
    ev = _ev(orc, w)

    def single_pixel_fraction(d):
        pix = orc.pixels(ev, d)
        owners = np.unique(w.owner[w.owner >= 0])
        single = sum(np.unique(pix[w.owner == o]).size == 1 for o in owners)
        return single / owners.size

    assert single_pixel_fraction(float(np.float32(w.spec.d_true))) >= 0.99
    assert single_pixel_fraction(0.2) < 0.3
    assert single_pixel_fraction(0.4) < 0.3


# ---------------------------------------------------------------- P5 bound

def _check_interval(orc, ev, d_a, d_b, ds):
    M = ev.M
    Sb, Nl, Hb = orc.bound(ev, d_a, d_b, want_image=True)
    Kb = orc.key(M, Sb, Nl)
    for d in ds:
        S, N, Hp = orc.point(ev, float(d), want_image=True)
        assert np.all(Hb >= Hp), (d_a, d_b, d)  # eq. (18)
        assert Nl <= N  # eq. (20) / supplement: mu_low <= mu
        assert Kb >= orc.key(M, S, N)  # eq. (15)-(16)
    return Kb


@pytest.mark.parametrize("cfg,foe", [("c1", None), ("c2", None), ("c2", (101.3, 57.85)),
                                     ("c1", (-20.5, 140.25))])
def test_bound_dominates_every_fp32_point(orc, cfg, foe):
    """Eq. (18) and (15)-(16): H_bar >= H pixelwise, N_low <= N and
    K_bar >= K for grid points and random fp32 d inside intervals of every
    size, including an off-grid FOE and one outside the image."""
    w = config_windows(cfg, [3], n_events=6000 if cfg == "c2" else 10_000)[0]
    s = w.spec
    ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, foe or s.foe)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    rng = np.random.default_rng(7)
    total = 0
    for depth in (0, 1, 3, 6, 9, 12, L - 2, L - 1):
        size = 1 << (L - depth)
        for _ in range(2):
            ja = int(rng.integers(0, (1 << depth))) * size
            jb = ja + size
            d_a = orc.grid_d(s.d_lo, s.d_hi, L, ja)
            d_b = orc.grid_d(s.d_lo, s.d_hi, L, jb)
            grid = [orc.grid_d(s.d_lo, s.d_hi, L, j)
                    for j in np.unique(np.linspace(ja, jb, min(size + 1, 9)).astype(np.int64))]
            ds = np.concatenate([grid, _f32_between(d_a, d_b, 40, rng)])
            total += ds.size
            _check_interval(orc, ev, d_a, d_b, ds)
    assert total >= 500


def test_bound_many_random_points_c1(orc):
    """Eq. (18) at 10^4 fp32 divergences in narrow and wide intervals."""
    w = config_windows("c1", [4], n_events=2000)[0]
    ev = _ev(orc, w)
    rng = np.random.default_rng(11)
    L = 14
    for depth in (2, 5, 8, 11, 13):
        size = 1 << (L - depth)
        ja = int(rng.integers(0, 1 << depth)) * size
        d_a = orc.grid_d(0.0, 1.0, L, ja)
        d_b = orc.grid_d(0.0, 1.0, L, ja + size)
        _check_interval(orc, ev, d_a, d_b, _f32_between(d_a, d_b, 2000, rng))


def test_bound_equals_point_at_singletons(orc):
    """Eq. (16)/(18): equality when the interval is a single value."""
    w = config_windows("c2", [5], n_events=20_000)[0]
    ev = _ev(orc, w)
    for d in (0.0, 0.013, 0.4, float(np.float32(w.spec.d_true)), 1.49):
        Sb, Nl, Hb = orc.bound(ev, d, d, want_image=True)
        S, N, Hp = orc.point(ev, d, want_image=True)
        assert (Sb, Nl) == (S, N) and np.array_equal(Hb, Hp)


@pytest.mark.parametrize("cfg,n,foe", [("c2", 30_000, None), ("c3", 20_000, None), ("c5", 20_000, None),
                                       ("c2", 20_000, (101.3, 57.85)), ("c1", 10_000, None)])
def test_n_low_is_the_in_image_count_at_the_far_end(orc, cfg, n, foe):
    """Eq. (12) moves every event away from the FOE as d grows (the warped
    coordinate is a monotone fp32 function of the rate, which grows with d),
    so an event inside the image at the far end of an interval is inside at
    the near end too: N_low of [d_a, d_b] (events inside at both ends) equals
    N of the point d_b.  Random intervals of every depth, and the range's
    ends."""
    w = config_windows(cfg, [3], n_events=n)[0]
    s = w.spec
    ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, foe or s.foe)
    rng = np.random.default_rng(17)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    for depth in sorted({0, 1, 2, 4, 7, 11, 15, L - 1} & set(range(L))):
        size = 1 << (L - depth)
        for _ in range(3):
            ja = int(rng.integers(0, 1 << depth)) * size
            d_a, d_b = orc.grid_d(s.d_lo, s.d_hi, L, ja), orc.grid_d(s.d_lo, s.d_hi, L, ja + size)
            _, n_low = orc.bound(ev, d_a, d_b)
            _, n_b = orc.point(ev, d_b)
            assert n_low == n_b, (cfg, depth, d_a, d_b)


def test_bound_valid_near_pixel_corners(orc):
    """Eq. (18) where fp32 rounding matters most: rays that pass within about
    an ulp of a pixel corner, probed at every fp32 d near the crossing.  The
    rounded warped point can land on either side of the corner, and the
    bound must still cover it."""
    W = H = 128
    cx = cy = 64.0
    tau = 0.5
    rng = np.random.default_rng(21)
    n = 400
    # a corner (X, Y) and a point on the FOE-corner ray, nudged sideways
    X = rng.integers(70, 120, n).astype(np.float64)
    Y = rng.integers(70, 120, n).astype(np.float64)
    frac = rng.uniform(0.55, 0.9, n)
    px = cx + (X - cx) * frac
    py = cy + (Y - cy) * frac
    x = px.astype(np.float32)
    y = py.astype(np.float32)
    t = rng.uniform(0.0, 0.2, n).astype(np.float32)
    misses = 0
    for i in range(n):
        ev = orc.Events(x[i:i + 1], y[i:i + 1], t[i:i + 1], tau, W, H, (cx, cy))
        delta = np.float32(tau) - t[i]
        ax = np.float32(np.float32(x[i] - np.float32(cx)) * delta)
        rc = (X[i] - float(x[i])) / float(ax)
        dc = rc / (1.0 + rc * tau)
        if not (0.0 < dc < 1.9):
            continue
        d_a, d_b = float(np.float32(dc * 0.98)), float(np.float32(min(dc * 1.02, 1.99)))
        _, _, Hb = orc.bound(ev, d_a, d_b, want_image=True)
        lo = np.array([dc * (1 - 2e-6)], np.float32).view(np.uint32)[0]
        hi = np.array([dc * (1 + 2e-6)], np.float32).view(np.uint32)[0]
        for bits in range(int(lo), int(hi) + 1):
            d = float(np.array([bits], np.uint32).view(np.float32)[0])
            p = orc.pixels(ev, d)[0]
            if p >= 0 and Hb[p] == 0:
                misses += 1
    assert misses == 0


def _pixel_segment_distance(px, py, ax0, ay0, bx0, by0):
    """Distance from the closed unit square [px, px+1] x [py, py+1] to the
    segment A-B (fp64; sampled finely along the segment)."""
    s = np.linspace(0.0, 1.0, 4001)
    X = ax0 + (bx0 - ax0) * s
    Y = ay0 + (by0 - ay0) * s
    dx = np.maximum(np.maximum(px - X, X - (px + 1)), 0.0)
    dy = np.maximum(np.maximum(py - Y, Y - (py + 1)), 0.0)
    return float(np.min(np.hypot(dx, dy)))


def test_walk_is_thin_single_events(orc):
    """Eq. (17) brute force, one event at a time: every pixel of H_bar lies
    within 2^-7 px of the segment joining the warped endpoints (the walk adds
    nothing far from the line), and the pixel of every sampled fp32 point of
    the interval is in H_bar."""
    w = config_windows("c1", [6], n_events=400)[0]
    s = w.spec
    rng = np.random.default_rng(3)
    L = 14
    for i in range(150):
        ev = orc.Events(w.x[i:i + 1], w.y[i:i + 1], w.t_rel[i:i + 1], s.tau, s.width, s.height, s.foe)
        depth = int(rng.integers(0, 10))
        size = 1 << (L - depth)
        ja = int(rng.integers(0, 1 << depth)) * size
        d_a, d_b = orc.grid_d(0, 1, L, ja), orc.grid_d(0, 1, L, ja + size)
        _, _, Hb = orc.bound(ev, d_a, d_b, want_image=True)
        xa, ya = npwarp.warp(ev.x, ev.y, ev.t, s.tau, s.foe[0], s.foe[1], d_a)
        xb, yb = npwarp.warp(ev.x, ev.y, ev.t, s.tau, s.foe[0], s.foe[1], d_b)
        for p in np.nonzero(Hb)[0]:
            dist = _pixel_segment_distance(p % s.width, p // s.width, float(xa[0]), float(ya[0]),
                                           float(xb[0]), float(yb[0]))
            assert dist <= 2.0 ** -7, (i, p, dist)
        for d in _f32_between(d_a, d_b, 30, rng):
            pix = orc.pixels(ev, float(d))[0]
            if pix >= 0:
                assert Hb[pix] == 1


# ---------------------------------------------------------------- P6 BnB

def test_bnb_equals_dense_sweep_c1(orc):
    """Algorithm 1 with exact keys returns the plain definition: the
    lexicographic max of (K_j, -j) over the grid (dense sweep)."""
    w = config_windows("c1", [0])[0]
    ev = _ev(orc, w)
    r = orc.bnb(ev, 0.0, 1.0, 1e-4)
    d = orc.dense(ev, 0.0, 1.0, 1e-4)
    assert r.status == 0 and (r.j_star, r.K) == (d.j_star, d.K)
    assert r.nodes_expanded < 200  # the bound prunes: far fewer than 2^14 - 1 points


@pytest.mark.parametrize("k", range(12))
def test_bnb_equals_dense_sweep_tiny(orc, k):
    w = config_windows("tiny", [k])[0]
    s = w.spec
    ev = _ev(orc, w)
    r = orc.bnb(ev, s.d_lo, s.d_hi, s.eps)
    d, S, N = orc.dense(ev, s.d_lo, s.d_hi, s.eps, want_all=True)
    assert (r.j_star, r.K) == (d.j_star, d.K)
    K = np.array([orc.key(ev.M, int(a), int(b)) for a, b in zip(S[1:-1], N[1:-1])], dtype=object)
    kmax = max(K)
    assert d.j_star == 1 + next(i for i, v in enumerate(K) if v == kmax)


@pytest.mark.parametrize("k", range(3))
def test_bnb_equals_dense_sweep_c2_shape(orc, k):
    w = config_windows("c2", [k], n_events=3000)[0]
    ev = _ev(orc, w)
    r = orc.bnb(ev, 0.0, 1.5, 1e-3)
    d = orc.dense(ev, 0.0, 1.5, 1e-3)
    assert (r.j_star, r.K) == (d.j_star, d.K)


def test_paper_mode_gamma_and_budget(orc):
    """Algorithm 1's stopping rule: with gamma > 0 the returned point is
    within gamma of the optimum in contrast; with a node budget the reported
    gap certifies the distance to the optimum."""
    w = config_windows("c1", [1])[0]
    ev = _ev(orc, w)
    M2 = float(ev.M) ** 2
    exact = orc.bnb(ev, 0.0, 1.0, 1e-4)
    for gamma in (0.025, 0.5, 3.0):
        r = orc.bnb(ev, 0.0, 1.0, 1e-4, gamma=gamma)
        assert r.status == 0
        assert (exact.K - r.K) / M2 <= gamma + 1e-12
        assert r.nodes_expanded <= exact.nodes_expanded
    b = orc.bnb(ev, 0.0, 1.0, 1e-4, max_nodes=5)
    assert b.status == orc.EBUDGET and b.nodes_expanded == 5
    assert b.gap * M2 >= (exact.K - b.K) - 1e-6 * M2


# ---------------------------------------------------------------- P7 continuum

@pytest.mark.parametrize("k", range(10))
def test_grid_optimum_against_continuum(orc, k):
    """Brute force over the continuum (tiny inputs): the contrast is constant
    between pixel-crossing breakpoints.  Every grid value that is not within
    rounding distance of a breakpoint equals its elementary interval's fp64
    value, so the grid optimum never exceeds the continuum optimum and equals
    it when the best elementary interval holds a grid point."""
    from oracle import continuum

    w = config_windows("tiny", [k])[0]
    s = w.spec
    ev = _ev(orc, w)
    cmax, bp, cmid = continuum.continuum_max(ev, s.d_lo, s.d_hi)
    d, S, N = orc.dense(ev, s.d_lo, s.d_hi, s.eps, want_all=True)
    L = d.L
    M2 = float(ev.M) ** 2
    js = np.arange(1, 1 << L)
    dj = np.array([orc.grid_d(s.d_lo, s.d_hi, L, int(j)) for j in js], np.float64)
    Cj = np.array([orc.key(ev.M, int(S[j]), int(N[j])) / M2 for j in js])
    cell = np.searchsorted(bp, dj, side="right") - 1
    cell = np.clip(cell, 0, cmid.size - 1)
    near = np.min(np.abs(dj[:, None] - bp[None, :]), axis=1) <= 1e-6
    far = ~near
    assert np.allclose(Cj[far], cmid[cell[far]], rtol=1e-12, atol=1e-12)
    assert d.contrast <= cmax + 1e-12 or near[d.j_star - 1]
    best_cells = np.nonzero(np.isclose(cmid, cmax, rtol=1e-12, atol=1e-12))[0]
    if np.any(np.isin(cell[far], best_cells)):
        assert d.contrast == pytest.approx(cmax, rel=1e-12)


# ---------------------------------------------------------------- P8 recovery

def test_recovers_true_divergence_noise_free(orc):
    """On noise-free descent the true D lies on the optimal plateau of the
    contrast, and the canonical optimum is the plateau's first grid point."""
    w = config_windows("noisefree", [0])[0]
    ev = _ev(orc, w)
    r = orc.bnb(ev, 0.0, 1.0, 1e-4)
    S, N = orc.point(ev, float(np.float32(0.3)))
    assert orc.key(ev.M, S, N) == r.K
    assert r.d_hat <= 0.3 and abs(r.d_hat - 0.3) < 1e-3
    for j in range(r.j_star, int(np.ceil(0.3 * (1 << 14)))):
        S, N = orc.point(ev, orc.grid_d(0, 1, 14, j))
        assert orc.key(ev.M, S, N) == r.K


@pytest.mark.parametrize("k", range(2))
def test_recovers_divergence_c2_noisy(orc, k):
    w = config_windows("c2", [k], n_events=30_000)[0]
    ev = _ev(orc, w)
    r = orc.bnb(ev, 0.0, 1.5, 1e-4)
    assert abs(r.d_hat - w.spec.d_true) < 0.02


# ---------------------------------------------------------------- grid, window

def test_grid_depth_and_points(orc):
    assert orc.depth(0.0, 1.0, 1e-4) == 14
    assert orc.depth(0.0, 1.5, 1e-5) == 18
    assert orc.depth(0.0, 2.0, 1e-5) == 18
    assert orc.grid_d(0.0, 1.0, 14, 1 << 13) == 0.5
    assert orc.grid_d(0.25, 1.25, 2, 3) == 1.0
    assert orc.rate(0.0, 0.5) == 0.0
    assert orc.rate(0.5, 0.5) == np.float32(0.5) / np.float32(0.75)


def test_window_selection_closed_interval(orc):
    t = np.array([0.9, 1.0, 1.2, 1.5, 1.5000001], np.float64)
    idx, tr = orc.select(t, 1.0, 1.5)
    assert list(idx) == [1, 2, 3]
    assert tr[0] == 0.0 and tr[2] == np.float32(0.5)


def test_downsample_matches_numpy(orc):
    """Input of the learned incumbent: unwarped counts on a 64x64 grid,
    scaled by 4096/N and rounded to bfloat16 (torch's round-to-nearest-even
    conversion is the reference rounding)."""
    import torch

    w = config_windows("c2", [0], n_events=50_000)[0]
    s = w.spec
    G = 64
    img = orc.downsample(w.x, w.y, s.width, s.height, G)
    bx = np.minimum(np.floor((w.x * np.float32(G)) / np.float32(s.width)), G - 1).astype(np.int64)
    by = np.minimum(np.floor((w.y * np.float32(G)) / np.float32(s.height)), G - 1).astype(np.int64)
    cnt = np.bincount(by * G + bx, minlength=G * G).astype(np.float32)
    v = cnt * (np.float32(G * G) / np.float32(w.n))
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(img.ravel(), ref)
