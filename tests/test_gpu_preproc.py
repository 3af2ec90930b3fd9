"""Preprocessing kernels (Sec. 6) against their CPU statement, bit for bit,
and estimation on the preprocessed windows."""

import numpy as np
import pytest

from synth import config_windows, pack_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2209_13168_amd import ecmd

    c = ecmd.Context(0)
    yield c
    c.close()


def test_hot_pixel_filter_bit_exact(ctx, orc):
    import dataclasses

    from oracle import preproc
    from paper_2209_13168_amd import ecmd
    from synth.ventral import make_window

    spec = dataclasses.replace(config_windows("c5", [0])[0].spec, n_events=60_000, n_points=3000)
    ws = [make_window(spec, 5, 500 + k) for k in range(3)]
    x, y, t, off, tau = pack_batch(ws)
    sen = ecmd.sensor(spec.width, spec.height, spec.foe)
    got = ctx.hot_pixel_filter(sen, x, y, t, off, 20)
    want = preproc.hot_pixel_filter(x, y, t, off, spec.width, spec.height, 20)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert got[3][-1] < off[-1] - 0.9 * sum(w.n_hot for w in ws)  # the hot pixels are gone
    # the filtered windows no longer lock onto d = 0 (hot pixels do not move)
    xo, yo, to, oo = got
    res = ctx.estimate_batched(sen, xo, yo, to, oo, tau, spec.d_lo, spec.d_hi, 1e-4)
    for r, w in zip(res, ws):
        assert abs(r.d_hat - w.spec.d_true) < 0.05, (r.d_hat, w.spec.d_true)


def test_resample_bit_exact_and_estimate(ctx, orc):
    from oracle import preproc
    from paper_2209_13168_amd import ecmd

    ws = config_windows("c2", range(3), n_events=40_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    sin = ecmd.sensor(s.width, s.height, s.foe)
    sout = ecmd.sensor(160, 90, (80.0, 45.0))
    got = ctx.resample(sin, sout, x, y, t, off, 0.25, 2209)
    want = preproc.resample(x, y, t, off, s.width, s.height, 160, 90, 0.25, 2209)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    xo, yo, to, oo = got
    res = ctx.estimate_batched(sout, xo, yo, to, oo, tau, s.d_lo, s.d_hi, 1e-4)
    for k, (r, w) in enumerate(zip(res, ws)):
        o = orc.bnb(orc.Events(xo[oo[k]:oo[k + 1]], yo[oo[k]:oo[k + 1]], to[oo[k]:oo[k + 1]], s.tau, 160, 90,
                               (80.0, 45.0)), s.d_lo, s.d_hi, 1e-4)
        assert (r.j_star, r.K) == (o.j_star, o.K)


def test_stream_windows_match_oracle(ctx, orc):
    """Stream mode (Sec. 4.4): a descent recorded as one stream, cut into
    consecutive windows; each window equals the oracle on the same events."""
    import torch

    from paper_2209_13168_amd import ecmd

    ws = config_windows("c2", range(4), n_events=15_000)
    s = ws[0].spec
    tau = float(np.float32(s.tau))
    t0 = 50.0
    t = np.concatenate([t0 + k * tau + w.t_rel.astype(np.float64) for k, w in enumerate(ws)])
    x = np.concatenate([w.x for w in ws])
    y = np.concatenate([w.y for w in ws])
    sen = ecmd.sensor(s.width, s.height, s.foe)
    host = ctx.estimate_stream(sen, x, y, t, t0, tau, len(ws), s.d_lo, s.d_hi, 1e-4)
    dev = torch.device("cuda:0")
    devr = ctx.estimate_stream(sen, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev),
                               torch.from_numpy(t).to(dev), t0, tau, len(ws), s.d_lo, s.d_hi, 1e-4)
    for k in range(len(ws)):
        lo, hi = t0 + k * tau, t0 + (k + 1) * tau
        sel = (t >= lo) & (t < hi)
        tr = (t[sel] - lo).astype(np.float32)
        o = orc.bnb(orc.Events(x[sel], y[sel], tr, tau, s.width, s.height, s.foe), s.d_lo, s.d_hi, 1e-4)
        for r in (host[k], devr[k]):
            assert r.status == 0 and (r.j_star, r.K) == (o.j_star, o.K)
            assert r.n_events == int(sel.sum())
