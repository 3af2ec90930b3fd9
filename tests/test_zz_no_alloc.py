"""The allocation-free batched search (``ecmd_estimate_divergence_batched_noalloc``).

It runs the asynchronous plan's search with every device buffer taken from
the library's static scratch array.  Two calls in a row, the second with
fewer and smaller windows, must each give the plan launch's results field
for field on the same input, and the oracle's canonical optimum; a call
whose buffers would not fit the array is refused before anything runs."""

import dataclasses

import numpy as np
import pytest

from synth import config_windows, pack_batch

pytestmark = pytest.mark.gpu

FIELDS = ("status", "j_star", "L", "d_hat", "K", "contrast", "d_end", "gap", "n_events", "nodes_expanded",
          "nodes_pruned", "point_evals", "bound_evals", "event_hyp_evals", "pixel_updates", "steps", "seeded")
EPS = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2209_13168_amd import ecmd

    assert torch.cuda.is_available()
    c = ecmd.Context(0)
    yield c
    c.close()


def _sensor(spec):
    from paper_2209_13168_amd import ecmd

    return ecmd.sensor(spec.width, spec.height, spec.foe)


def _dev(*arrs):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _windows(ns, seed):
    from synth.ventral import make_window

    ws = config_windows("c2", range(len(ns)))
    return [make_window(dataclasses.replace(w.spec, n_events=n), 2, seed + i) for i, (w, n) in enumerate(zip(ws, ns))]


def _noalloc(ctx, spec, arrs, max_events):
    import torch

    from paper_2209_13168_amd.ecmd import BatchPlan

    B = int(arrs[4].shape[0])
    out = BatchPlan.result_buffer(B)
    ctx.estimate_batched_noalloc(_sensor(spec), *arrs, spec.d_lo, spec.d_hi, EPS, max_events, out)
    torch.cuda.synchronize()
    return BatchPlan.results(out, B)


def _planned(ctx, spec, arrs, max_events):
    import torch

    B = int(arrs[4].shape[0])
    plan = ctx.batch_plan(_sensor(spec), spec.d_lo, spec.d_hi, EPS, max_windows=B, max_events=max_events)
    out = plan.result_buffer(B)
    plan.launch(*arrs, out)
    torch.cuda.synchronize()
    res = plan.results(out, B)
    plan.close()
    return res


@pytest.mark.parametrize("ns,seed", [((0, 1, 500, 3000, 9000, 40_000), 700), ((2000, 15_000, 7), 800)])
def test_noalloc_equals_the_plan_launch_and_the_oracle(ctx, orc, ns, seed):
    """Both parametrisations run in one process, one after the other: the
    second call finds the first call's contents in the scratch."""
    wins = _windows(ns, seed)
    s = wins[0].spec
    x, y, t, off, tau = pack_batch(wins)
    arrs = _dev(x, y, t, off, tau)
    max_events = int(off[-1]) + 17
    got = _noalloc(ctx, s, arrs, max_events)
    ref = _planned(ctx, s, arrs, max_events)
    for i, w in enumerate(wins):
        for f in FIELDS:
            assert getattr(got[i], f) == getattr(ref[i], f), (i, f, got[i], ref[i])
        o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, EPS)
        assert (got[i].status, got[i].j_star, got[i].K) == (0, o.j_star, o.K), (i, got[i], o)
    # the same input again: the scratch holds this call's own last contents
    again = _noalloc(ctx, s, arrs, max_events)
    for a, b in zip(again, got):
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), (f, a, b)


def test_noalloc_two_calls_second_smaller(ctx, orc):
    big = _windows((3000, 25_000, 9000, 120, 60_000), 900)
    small = _windows((4000, 50), 950)
    s = big[0].spec
    for wins in (big, small):
        x, y, t, off, tau = pack_batch(wins)
        arrs = _dev(x, y, t, off, tau)
        got = _noalloc(ctx, s, arrs, int(off[-1]))
        ref = _planned(ctx, s, arrs, int(off[-1]))
        for i, w in enumerate(wins):
            for f in FIELDS:
                assert getattr(got[i], f) == getattr(ref[i], f), (i, f, got[i], ref[i])
            o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, EPS)
            assert (got[i].j_star, got[i].K) == (o.j_star, o.K), (i, got[i], o)


def test_noalloc_refuses_what_the_scratch_cannot_hold(ctx):
    from paper_2209_13168_amd import ecmd

    wins = _windows((1000, 2000), 990)
    s = wins[0].spec
    x, y, t, off, tau = pack_batch(wins)
    arrs = _dev(x, y, t, off, tau)
    # 2^24 events need 2^24 x 16 B x 2 tiles of one FOE quadrant = 512 MiB of event store
    with pytest.raises(ecmd.EcmdError) as err:
        _noalloc(ctx, s, arrs, 1 << 24)
    assert err.value.code == ecmd.ENOMEM and "scratch" in str(err.value)
    # the refused call launched nothing: a fitting call right after is exact
    got = _noalloc(ctx, s, arrs, int(off[-1]))
    ref = _planned(ctx, s, arrs, int(off[-1]))
    for a, b in zip(got, ref):
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), (f, a, b)
