"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work (pixel indices, counts, sums of squares, contrast keys, grid
indices) must match bit for bit.  Inputs come from the seeded generator and
are passed to both sides unchanged.
"""

import numpy as np
import pytest

from synth import config_windows, pack_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2209_13168_amd import ecmd

    assert torch.cuda.is_available()
    c = ecmd.Context(0)
    yield c
    c.close()


def _sensor(spec, foe=None):
    from paper_2209_13168_amd import ecmd

    return ecmd.sensor(spec.width, spec.height, foe or spec.foe)


def _f32_between(lo, hi, n, rng):
    a = np.array([lo], np.float32).view(np.uint32)[0]
    b = np.array([hi], np.float32).view(np.uint32)[0]
    return rng.integers(int(a), int(b) + 1, n, dtype=np.int64).astype(np.uint32).view(np.float32)


CASES = [
    ("c1", {}, None),
    ("c2", {"n_events": 30_000}, None),
    ("c2", {"n_events": 8_000}, (101.3, 57.85)),
    ("c3", {"n_events": 60_000}, None),
    ("c3", {"n_events": 30_000}, (300.5, 200.25)),
]


@pytest.mark.parametrize("cfg,kw,foe", CASES)
def test_pixels_bit_exact(ctx, orc, cfg, kw, foe):
    w = config_windows(cfg, [0], **kw)[0]
    s = w.spec
    ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, foe or s.foe)
    rng = np.random.default_rng(5)
    for d in list(_f32_between(s.d_lo, s.d_hi, 6, rng)) + [0.0, np.float32(s.d_true)]:
        got = ctx.probe_pixels(_sensor(s, foe), w.x, w.y, w.t_rel, s.tau, float(d))
        assert np.array_equal(got, orc.pixels(ev, float(d))), d


@pytest.mark.parametrize("cfg,kw,foe", CASES)
def test_point_values_bit_exact(ctx, orc, cfg, kw, foe):
    w = config_windows(cfg, [1], **kw)[0]
    s = w.spec
    ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, foe or s.foe)
    rng = np.random.default_rng(6)
    ds = np.concatenate([_f32_between(s.d_lo, s.d_hi, 13, rng), [0.0, np.float32(s.d_true)]]).astype(np.float32)
    S, N, img = ctx.probe_point(_sensor(s, foe), w.x, w.y, w.t_rel, s.tau, ds, want_image=True)
    M = s.width * s.height
    for k, d in enumerate(ds):
        So, No, Ho = orc.point(ev, float(d), want_image=True)
        assert (int(S[k]), int(N[k])) == (So, No), (k, d)
        assert np.array_equal(img[k * M:(k + 1) * M], Ho)


@pytest.mark.parametrize("cfg,kw,foe", CASES)
def test_bound_values_bit_exact(ctx, orc, cfg, kw, foe):
    w = config_windows(cfg, [2], **kw)[0]
    s = w.spec
    ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, foe or s.foe)
    L = orc.depth(s.d_lo, s.d_hi, s.eps)
    rng = np.random.default_rng(7)
    da, db = [], []
    for depth in (0, 1, 2, 4, 7, 10, 13, L - 1):
        size = 1 << (L - depth)
        ja = int(rng.integers(0, 1 << depth)) * size
        da.append(orc.grid_d(s.d_lo, s.d_hi, L, ja))
        db.append(orc.grid_d(s.d_lo, s.d_hi, L, ja + size))
    d = float(np.float32(s.d_true))
    da.append(d)
    db.append(d)  # singleton
    da = np.array(da, np.float32)
    db = np.array(db, np.float32)
    Sb, Nl, img = ctx.probe_bound(_sensor(s, foe), w.x, w.y, w.t_rel, s.tau, s.d_lo, s.d_hi, da, db,
                                  want_image=True)
    M = s.width * s.height
    for k in range(da.size):
        So, No, Ho = orc.bound(ev, float(da[k]), float(db[k]), want_image=True)
        assert (int(Sb[k]), int(Nl[k])) == (So, No), (k, da[k], db[k])
        assert np.array_equal(img[k * M:(k + 1) * M], Ho)


def _check_same(r, o):
    assert r.status == 0, r
    assert (r.j_star, r.K) == (o.j_star, o.K), (r, o)
    assert r.d_hat == o.d_hat


@pytest.mark.parametrize("k", range(3))
def test_bnb_c1_single_window(ctx, orc, k):
    """Canonical optimum of Algorithm 1 on the 128x128 config, single-window
    entry point (absolute fp64 times, window selection on the device)."""
    import torch

    w = config_windows("c1", [k])[0]
    s = w.spec
    o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
    r = ctx.estimate(_sensor(s), w.x, w.y, w.t, s.t0, w.t1, s.d_lo, s.d_hi, s.eps)
    _check_same(r, o)
    dev = torch.device("cuda:0")
    rd = ctx.estimate(_sensor(s), torch.from_numpy(w.x).to(dev), torch.from_numpy(w.y).to(dev),
                      torch.from_numpy(w.t).to(dev), s.t0, w.t1, s.d_lo, s.d_hi, s.eps)
    _check_same(rd, o)
    assert r.nodes_expanded > 0 and r.event_hyp_evals > 0


@pytest.mark.parametrize("k", range(2))
def test_bnb_c2_full_window(ctx, orc, k):
    """346x260 sensor, 100k events, eps 1e-5 (depth 18)."""
    w = config_windows("c2", [k])[0]
    s = w.spec
    o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
    x, y, t, off, tau = pack_batch([w])
    r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)[0]
    _check_same(r, o)


def test_bnb_batched_mixed_sizes(ctx, orc):
    """Windows of very different sizes in one batched call, each equal to
    its own oracle optimum; frontier batch sizes 1, 8, 64 agree."""
    ws = config_windows("c2", range(6))
    ns = [0, 1, 500, 3000, 9000, 20_000]
    import dataclasses

    from synth.ventral import make_window

    wins = [make_window(dataclasses.replace(w.spec, n_events=n), 2, 100 + i) for i, (w, n) in enumerate(zip(ws, ns))]
    s = wins[0].spec
    x, y, t, off, tau = pack_batch(wins)
    outs = {}
    for F in (1, 8, 64):
        outs[F] = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4, frontier_batch=F)
    for i, wv in enumerate(wins):
        o = orc.bnb(orc.Events.of_window(wv), s.d_lo, s.d_hi, 1e-4)
        for F in outs:
            _check_same(outs[F][i], o)


@pytest.mark.parametrize("k", range(8))
def test_bnb_tiny_windows(ctx, orc, k):
    w = config_windows("tiny", [k])[0]
    s = w.spec
    o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
    d = orc.dense(orc.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
    assert (o.j_star, o.K) == (d.j_star, d.K)
    x, y, t, off, tau = pack_batch([w])
    r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)[0]
    _check_same(r, o)


def test_seeds_do_not_change_the_optimum(ctx, orc):
    ws = config_windows("c2", range(4), n_events=15_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    plain = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
    seeds = np.array([w.spec.d_true for w in ws], np.float32)
    seeds[1] = np.nan  # no seed for this window
    seeds[2] = 1.49  # a bad seed
    seeded = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4, d_seeds=seeds)
    for i, w in enumerate(ws):
        o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, 1e-4)
        _check_same(plain[i], o)
        _check_same(seeded[i], o)
    assert seeded[0].seeded == 1 and seeded[1].seeded == 0


def test_paper_mode_gamma_and_budget(ctx, orc):
    w = config_windows("c1", [1])[0]
    s = w.spec
    ev = orc.Events.of_window(w)
    exact = orc.bnb(ev, s.d_lo, s.d_hi, s.eps)
    M2 = float(s.width * s.height) ** 2
    x, y, t, off, tau = pack_batch([w])
    for gamma in (0.025, 0.5):
        r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, gamma=gamma)[0]
        assert r.status == 0
        assert (exact.K - r.K) / M2 <= gamma + 1e-12
        S, N = orc.point(ev, r.d_hat)
        assert orc.key(ev.M, S, N) == r.K
    from paper_2209_13168_amd import ecmd

    b = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, max_nodes=5,
                             frontier_batch=2)[0]
    assert b.status == ecmd.EBUDGET
    assert b.nodes_expanded <= 5
    assert b.gap * M2 >= (exact.K - b.K) - 1e-6 * M2
    S, N = orc.point(ev, b.d_hat)
    assert orc.key(ev.M, S, N) == b.K


def test_edge_cases(ctx, orc):
    """No events, one event, events at t = tau, events on the FOE."""
    spec = config_windows("c1", [0])[0].spec
    W, H = spec.width, spec.height
    cases = [
        (np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32)),
        (np.array([10.5], np.float32), np.array([99.25], np.float32), np.array([0.1], np.float32)),
        (np.full(7, 30.0, np.float32), np.full(7, 40.0, np.float32), np.full(7, 0.5, np.float32)),
        (np.full(5, 64.0, np.float32), np.full(5, 64.0, np.float32), np.linspace(0, 0.5, 5).astype(np.float32)),
    ]
    M2 = float(W * H) ** 2
    for x, y, t in cases:
        ev = orc.Events(x, y, t, 0.5, W, H, spec.foe)
        o = orc.bnb(ev, 0.0, 1.0, 1e-3)
        r = ctx.estimate_batched(_sensor(spec), x, y, t, np.array([0, x.size], np.int64),
                                 np.array([0.5], np.float32), 0.0, 1.0, 1e-3)[0]
        _check_same(r, o)
        # the gamma stop (with certified children): gamma-optimal, the gap covering the loss
        g = ctx.estimate_batched(_sensor(spec), x, y, t, np.array([0, x.size], np.int64),
                                 np.array([0.5], np.float32), 0.0, 1.0, 1e-3, gamma=0.025)[0]
        assert g.status == 0 and 0.0 <= (o.K - g.K) / M2 <= g.gap <= 0.025, (g, o)
        S, N = orc.point(ev, g.d_hat)
        assert orc.key(ev.M, S, N) == g.K


def test_invalid_arguments_rejected(ctx):
    from paper_2209_13168_amd import ecmd

    spec = config_windows("c1", [0])[0].spec
    x = np.array([1.0], np.float32)
    off = np.array([0, 1], np.int64)
    tau = np.array([0.5], np.float32)
    bad = [
        dict(t=np.array([0.7], np.float32), lo=0.0, hi=1.0, eps=1e-3),  # t' > tau
        dict(t=np.array([0.1], np.float32), lo=0.0, hi=2.0, eps=1e-3),  # d_hi * tau >= 1
        dict(t=np.array([0.1], np.float32), lo=0.5, hi=0.5, eps=1e-3),  # empty range
        dict(t=np.array([0.1], np.float32), lo=0.0, hi=1.0, eps=0.0),  # eps
        dict(t=np.array([np.nan], np.float32), lo=0.0, hi=1.0, eps=1e-3),  # NaN time
    ]
    for b in bad:
        with pytest.raises(ecmd.EcmdError) as e:
            ctx.estimate_batched(_sensor(spec), x, x, b["t"], off, tau, b["lo"], b["hi"], b["eps"])
        assert e.value.code == ecmd.EINVAL


def test_downsample_bit_exact(ctx, orc):
    ws = config_windows("c2", range(3), n_events=20_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    got = ctx.downsample(_sensor(s), x, y, off).reshape(len(ws), 64, 64)
    for i, w in enumerate(ws):
        assert np.array_equal(got[i], orc.downsample(w.x, w.y, s.width, s.height))


def test_graph_replay_and_tunings_match(ctx, orc):
    """The captured step graph, replayed across several calls with eager
    calls in between, and every tuning the autotuner may pick, give the
    oracle's optima."""
    ws = config_windows("c2", range(5), n_events=12_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    sen = _sensor(s)
    want = [orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, 1e-4) for w in ws]
    saved = ctx.tuning()
    try:
        for F, tile, graph, group in [(64, 0, True, 0), (16, 0, True, 3), (64, 11000, False, 0),
                                      (128, 6000, True, 8), (64, 0, False, 1), (64, 0, True, 0)]:
            ctx.set_tuning(F, tile, graph, group)
            for _ in range(2):
                got = ctx.estimate_batched(sen, x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
                for r, o in zip(got, want):
                    _check_same(r, o)
        best = ctx.autotune(sen, x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
        assert best["frontier_batch"] in (16, 32, 96, 128, 256)
        got = ctx.estimate_batched(sen, x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
        for r, o in zip(got, want):
            _check_same(r, o)
    finally:
        ctx.set_tuning(**saved)


@pytest.mark.parametrize("tile,nt", [(0, 256), (0, 512), (0, 1024), (7000, 256), (9000, 512), (13000, 1024)])
def test_workgroup_sizes_and_tilings_bit_exact(ctx, orc, tile, nt):
    """Every evaluation workgroup size, on whole-LDS and on smaller tiles
    (guest copies, bordered counters at every cut), gives the oracle's point
    and bound values and optima."""
    saved = ctx.tuning()
    try:
        ctx.set_tuning(tile_px=tile, eval_threads=nt)
        assert ctx.tuning()["eval_threads"] == nt
        w = config_windows("c3", [4], n_events=30_000)[0]
        s = w.spec
        ev = orc.Events(w.x, w.y, w.t_rel, s.tau, s.width, s.height, s.foe)
        ds = np.array([0.0, 0.2, np.float32(s.d_true), 1.1, 1.45], np.float32)
        S, N = ctx.probe_point(_sensor(s), w.x, w.y, w.t_rel, s.tau, ds)[:2]
        for k, d in enumerate(ds):
            assert (int(S[k]), int(N[k])) == orc.point(ev, float(d))[:2], (k, d)
        L = orc.depth(s.d_lo, s.d_hi, s.eps)
        da = np.array([orc.grid_d(s.d_lo, s.d_hi, L, j) for j in (0, 1 << (L - 1), 3 << (L - 3))], np.float32)
        db = np.array([orc.grid_d(s.d_lo, s.d_hi, L, j) for j in (1 << L, 3 << (L - 2), (3 << (L - 3)) + 7)],
                      np.float32)
        Sb, Nl = ctx.probe_bound(_sensor(s), w.x, w.y, w.t_rel, s.tau, s.d_lo, s.d_hi, da, db)[:2]
        for k in range(da.size):
            assert (int(Sb[k]), int(Nl[k])) == orc.bound(ev, float(da[k]), float(db[k]))[:2], k
        ws = config_windows("c2", range(3), n_events=8_000)
        s2 = ws[0].spec
        x, y, t, off, tau = pack_batch(ws)
        got = ctx.estimate_batched(_sensor(s2), x, y, t, off, tau, s2.d_lo, s2.d_hi, 1e-4)
        for r, wv in zip(got, ws):
            _check_same(r, orc.bnb(orc.Events.of_window(wv), s2.d_lo, s2.d_hi, 1e-4))
    finally:
        ctx.set_tuning(**saved)


def test_search_is_reproducible(ctx):
    """Node counts, steps and pixel counts are identical call after call (the
    frontier step orders everything by scans, not by atomic races)."""
    ws = config_windows("c2", range(3), n_events=20_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    runs = [ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4) for _ in range(10)]
    key = lambda rs: [(r.j_star, r.K, r.nodes_expanded, r.bound_evals, r.pixel_updates, r.steps) for r in rs]
    assert all(key(r) == key(runs[0]) for r in runs[1:])


def test_profiling_timers(ctx):
    """The per-phase timers (kernel times taken from each launch's own
    dispatch): every evaluation launch pairs with a frontier launch, the
    times are positive and fit inside the calls' wall time, a reset clears
    them, and timing the kernels changes no result."""
    import time

    ws = config_windows("c2", range(4), n_events=20_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    key = lambda rs: [(r.j_star, r.K, r.nodes_expanded, r.bound_evals, r.pixel_updates, r.steps) for r in rs]
    ref = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
    ctx.set_profiling(True)
    try:
        ctx.profile(reset=True)
        t0 = time.perf_counter()
        runs = [ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4) for _ in range(3)]
        wall_ms = (time.perf_counter() - t0) * 1e3
        p = ctx.profile(reset=True)
        cleared = ctx.profile()
    finally:
        ctx.set_profiling(False)
    assert all(key(r) == key(ref) for r in runs)
    assert p["calls"] == 3
    assert p["eval_launches"] >= 3 * max(r.steps for r in ref)
    assert p["frontier_launches"] == p["eval_launches"]
    assert p["eval_ms"] > 0 and p["frontier_ms"] > 0 and p["prep_ms"] > 0
    assert p["eval_ms"] + p["frontier_ms"] + p["prep_ms"] < wall_ms
    assert cleared["calls"] == 0 and cleared["eval_launches"] == 0 and cleared["eval_ms"] == 0.0
    # off again: nothing is accumulated
    ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
    assert ctx.profile()["calls"] == 0


def test_measured_peaks_are_plausible(ctx):
    """The calibration kernels run and give rates within the chip's reach
    (LDS atomic adds under 64 lanes per cycle x 2.4 GHz x 256 CUs; HBM read
    under the 8 TB/s specification)."""
    p = ctx.measure_peaks(1 << 30)
    assert 1e11 < p["lds_atomics_per_s"] < 256 * 64 * 2.4e9 * 1.05
    assert 5e11 < p["hbm_read_bytes_per_s"] < 8.2e12


def test_host_plan_matches_the_device_search(ctx):
    """ecmd_plan (host only) gives the grid depth the device search uses."""
    from paper_2209_13168_amd import ecmd

    w = config_windows("c2", [5], n_events=5000)[0]
    s = w.spec
    x, y, t, off, tau = pack_batch([w])
    r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)[0]
    p = ecmd.plan(_sensor(s), s.d_lo, s.d_hi, s.eps)
    assert r.L == p["L"] and (p["segments"], p["eval_threads"]) == (8, 512)
    assert r.d_hat == np.float32(ecmd.grid_point(s.d_lo, s.d_hi, p["L"], r.j_star))
