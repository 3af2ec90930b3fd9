"""The device frontier (Algorithm 1) against the oracle's serial search.

With one node per step the frontier must pop exactly the node Algorithm 1
pops (the largest bound, ties to the smaller grid index), so the whole
expansion sequence, and with it every counter, equals the oracle's serial
best-first search; in paper mode (gamma stop) the returned grid point then
equals the oracle's too.  A frontier that outgrows its capacity stops that
window with ECMD_EFRONTIER, an uncertified incumbent (gap = infinity) whose
key is still exact, and leaves the other windows of the batch untouched.
"""

import dataclasses

import numpy as np
import pytest

from synth import config_windows, pack_batch
from synth.ventral import make_window

pytestmark = pytest.mark.gpu


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


def _windows():
    ws = config_windows("c1", range(3))
    ws += config_windows("tiny", range(4))
    c2 = config_windows("c2", [3], n_events=20_000)[0]
    return ws, c2


def _same_sequence(r, o):
    # the oracle evaluates the root centre once more (its initial incumbent)
    # and bounds the root interval, which the device never needs
    assert r.status == 0, r
    assert (r.j_star, r.K) == (o.j_star, o.K), (r, o)
    assert r.nodes_expanded == o.nodes_expanded, (r.nodes_expanded, o.nodes_expanded)
    assert r.point_evals + 1 == o.point_evals, (r.point_evals, o.point_evals)
    assert r.bound_evals + 1 == o.bound_evals, (r.bound_evals, o.bound_evals)


def test_one_node_per_step_is_algorithm1(ctx, orc):
    ws, c2 = _windows()
    for w in ws + [c2]:
        s = w.spec
        eps = s.eps if w is not c2 else 1e-4
        x, y, t, off, tau = pack_batch([w])
        r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, eps, frontier_batch=1)[0]
        o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, eps)
        _same_sequence(r, o)
        assert r.steps == r.nodes_expanded - 1  # one node per step after the root


@pytest.mark.parametrize("gamma", [0.025, 0.1])
def test_one_node_per_step_gamma_stop_is_algorithm1(ctx, orc, gamma):
    """Paper mode: the first pop whose bound is within gamma of the
    incumbent ends the search, on both sides at the same node."""
    for k in range(3):
        w = config_windows("c1", [k])[0]
        s = w.spec
        x, y, t, off, tau = pack_batch([w])
        r = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, gamma=gamma,
                                 frontier_batch=1)[0]
        o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, s.eps, gamma=gamma)
        assert r.status == 0
        assert (r.j_star, r.K, r.nodes_expanded) == (o.j_star, o.K, o.nodes_expanded), (r, o)


def test_frontier_overflow(ctx, orc):
    from paper_2209_13168_amd import ecmd

    big = config_windows("c1", [0])[0]
    s = big.spec
    # a window whose events sit at the FOE never moves: its contrast is the
    # same at every d, so ties leave one queued node per step
    still = make_window(dataclasses.replace(s, n_events=0), 1, 7)
    still = dataclasses.replace(still, x=np.full(5, s.foe[0], np.float32), y=np.full(5, s.foe[1], np.float32),
                                t_rel=np.linspace(0, 0.4, 5).astype(np.float32), p=np.ones(5, np.int8),
                                owner=np.full(5, -1, np.int32))
    x, y, t, off, tau = pack_batch([big, still])
    rs = ctx.estimate_batched(_sensor(s), x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, frontier_capacity=3)
    r0, r1 = rs
    assert r0.status == ecmd.EFRONTIER, r0
    assert r0.gap == float("inf")
    ev = orc.Events.of_window(big)
    S, N = orc.point(ev, r0.d_hat)
    assert orc.key(ev.M, S, N) == r0.K
    assert r0.d_hat == orc.grid_d(s.d_lo, s.d_hi, r0.L, r0.j_star)
    o1 = orc.bnb(orc.Events.of_window(still), s.d_lo, s.d_hi, s.eps)
    assert r1.status == 0 and (r1.j_star, r1.K) == (o1.j_star, o1.K), (r1, o1)
    # the same window alone with the default capacity is certified
    ok = ctx.estimate_batched(_sensor(s), *pack_batch([big]), s.d_lo, s.d_hi, s.eps)[0]
    o0 = orc.bnb(ev, s.d_lo, s.d_hi, s.eps)
    assert ok.status == 0 and (ok.j_star, ok.K) == (o0.j_star, o0.K)
    assert r0.K <= o0.K
