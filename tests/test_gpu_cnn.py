"""The learned-incumbent network on the GPU against its CPU statement."""

import numpy as np
import pytest

from synth import config_windows, pack_batch
from tests.test_oracle_cnn import _rand

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2209_13168_amd import ecmd

    c = ecmd.Context(0)
    yield c
    c.close()


def test_forward_matches_cpu_statement(ctx):
    from oracle import cnn as ocnn
    from paper_2209_13168_amd import ecmd

    net = ecmd.Cnn(ctx, seed=3)
    for seed in (0, 1):
        p, x, _ = _rand(seed, B=16)
        net.set_params(p)
        got = net.forward(x.reshape(16, -1))
        want = ocnn.predict(p, x)
        assert np.allclose(got, want, rtol=5e-3, atol=2e-3), np.abs(got - want).max()
    net.close()


@pytest.mark.parametrize("seed", [5, 6])
def test_gradients_match_cpu_statement(ctx, seed):
    """Every element of the batch gradient (bfloat16 layer inputs, fp32 sums)
    against the fp64 statement with the same roundings:
    |g - g64| <= 2^-7 |g64| + 2^-9 max|g64| per layer.  The two sides round the
    same layer inputs to bfloat16; where an fp32 activation and its fp64
    counterpart fall on either side of a rounding boundary the input differs
    by one bfloat16 step (2^-7 relative), which moves a gradient element by at
    most 2^-7 of its terms' magnitude: the relative term covers elements
    without cancellation, the absolute one (a share of the layer's largest
    element) those whose terms cancel.  The per-layer norm is checked too."""
    from oracle import cnn as ocnn
    from paper_2209_13168_amd import ecmd

    net = ecmd.Cnn(ctx, seed=4)
    p, x, y = _rand(seed, B=8)
    net.set_params(p)
    g, loss = net.grads(x.reshape(8, -1), y)
    loss_o, g_o, _ = ocnn.loss_and_grad(p, x, y, rounding=True)
    assert loss == pytest.approx(loss_o, rel=1e-2)
    k = 0
    worst = {}
    for name, shape in ocnn.SHAPES:
        n = int(np.prod(shape))
        a, b = g[k:k + n].astype(np.float64), g_o[k:k + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 1e-2, (name, rel)
        tol = 2.0**-7 * np.abs(b) + 2.0**-9 * np.abs(b).max()
        excess = np.abs(a - b) / np.maximum(tol, 1e-30)
        worst[name] = float(excess.max())
        bad = np.flatnonzero(np.abs(a - b) > tol)
        assert bad.size == 0, (name, bad[:8], a[bad[:8]], b[bad[:8]])
        k += n
    assert k == ecmd.CNN_NPARAM
    print("largest |g - g64| / tolerance per layer:", {k: round(v, 3) for k, v in worst.items()})
    net.close()


def test_training_reduces_the_loss(ctx):
    from paper_2209_13168_amd import ecmd

    ws = config_windows("c4", range(64), n_events=20_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    imgs = ctx.downsample(ecmd.sensor(s.width, s.height, s.foe), x, y, off).reshape(len(ws), -1)
    labels = np.array([w.spec.d_true for w in ws], np.float32)
    net = ecmd.Cnn(ctx, seed=7)
    first = net.train_step(imgs, labels, 1e-3)
    for _ in range(150):
        last = net.train_step(imgs, labels, 1e-3)
    assert last < 0.5 * first, (first, last)
    net.close()


def test_checkpoint_resumes_training_exactly(ctx, tmp_path):
    """Parameters and Adam state saved mid-training and loaded into another
    network continue the same trajectory bit for bit; a damaged file is
    rejected and leaves the network as it was."""
    from paper_2209_13168_amd import ecmd

    p, x, y = _rand(9, B=8)
    imgs = x.reshape(8, -1)
    a = ecmd.Cnn(ctx, seed=1)
    a.set_params(p)
    for _ in range(3):
        a.train_step(imgs, y, 1e-3)
    ck = str(tmp_path / "net.ckpt")
    a.save(ck)
    for _ in range(2):
        a.train_step(imgs, y, 1e-3)
    b = ecmd.Cnn(ctx, seed=2)
    b.load(ck)
    for _ in range(2):
        b.train_step(imgs, y, 1e-3)
    assert np.array_equal(a.params().view(np.uint32), b.params().view(np.uint32))
    raw = open(ck, "rb").read()
    assert raw[:8] == b"ECMDCNN1" and len(raw) == 16 + 3 * 4 * ecmd.CNN_NPARAM
    before = b.params()
    for bad in (b"XCMDCNN1" + raw[8:], raw[:-4], raw + b"\0"):
        open(ck, "wb").write(bad)
        with pytest.raises(ecmd.EcmdError):
            b.load(ck)
    assert np.array_equal(before.view(np.uint32), b.params().view(np.uint32))
    with pytest.raises(ecmd.EcmdError):
        b.load(str(tmp_path / "missing.ckpt"))
    a.close()
    b.close()


def test_learned_seeding_keeps_the_certified_optimum(ctx, orc):
    from paper_2209_13168_amd import ecmd

    ws = config_windows("c4", range(1_000_000, 1_000_004), n_events=15_000)
    s = ws[0].spec
    x, y, t, off, tau = pack_batch(ws)
    sen = ecmd.sensor(s.width, s.height, s.foe)
    net = ecmd.Cnn(ctx, seed=1)
    learned = ctx.estimate_learned(net, sen, x, y, t, off, tau, s.d_lo, s.d_hi, 1e-4)
    for w, r in zip(ws, learned):
        o = orc.bnb(orc.Events.of_window(w), s.d_lo, s.d_hi, 1e-4)
        assert r.status == 0 and (r.j_star, r.K) == (o.j_star, o.K)
        assert r.seeded == 1
    net.close()


def test_network_outliving_its_context_is_rejected_not_used():
    """Destroying a context releases its networks' device memory; the
    orphaned handle then rejects every call except destroy."""
    import ctypes as C

    from paper_2209_13168_amd import ecmd

    c = ecmd.Context(0)
    net = ecmd.Cnn(c, seed=3)
    h = net.h
    c.close()
    p = np.zeros(ecmd.CNN_NPARAM, np.float32)
    assert ecmd.lib().ecmd_cnn_get_params(h, p.ctypes.data) == ecmd.EINVAL
    assert ecmd.lib().ecmd_cnn_set_params(h, p.ctypes.data) == ecmd.EINVAL
    out = np.zeros(1, np.float32)
    img = np.zeros(4096, np.uint16)
    assert ecmd.lib().ecmd_cnn_forward(h, img.ctypes.data, 1, 0, out.ctypes.data) == ecmd.EINVAL
    assert ecmd.lib().ecmd_cnn_train_step(h, img.ctypes.data, out.ctypes.data, 1, C.c_float(1e-3), 0, None) == ecmd.EINVAL
    net.close()  # frees the empty handle
    assert net.h is None


def test_trained_network_gains_on_held_out_windows(ctx):
    """The committed proposal network on held-out 346x260 windows (never
    trained on): its error against the certified optimum beats a constant
    guess by a wide margin; the certified optimum is the same with and without
    its seeds; the seeds save node expansions both in the canonical search and
    with Algorithm 1's gamma stop of Sec. 6 (deterministic: same windows, same
    weights); and the network's forward pass costs under 2% of the seeded
    search."""
    import os
    import time

    import torch

    from paper_2209_13168_amd import ecmd, learned

    path = os.path.join(os.path.dirname(learned.__file__), "weights", "cnn_c2.npz")
    assert os.path.exists(path), "trained weights are missing"
    net, meta = learned.load(ctx, path)
    wins = config_windows("c4", range(learned.HELD_OUT + 5000, learned.HELD_OUT + 5064))
    s = wins[0].spec
    dev = torch.device("cuda:0")
    x, y, t, off, tau = (torch.from_numpy(a).to(dev) for a in pack_batch(wins))
    sen = ecmd.sensor(*learned.SENSOR)
    plain = ctx.estimate_batched(sen, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)
    seeded = ctx.estimate_learned(net, sen, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)
    assert [(r.j_star, r.K) for r in plain] == [(r.j_star, r.K) for r in seeded]
    assert all(r.seeded == 1 for r in seeded)
    imgs = ctx.downsample(sen, x, y, off).cpu().numpy().view(np.uint16).reshape(len(wins), -1)
    pred = net.forward(imgs)
    lab = np.array([r.d_hat for r in plain])
    err = np.abs(pred - lab).mean()
    const = np.abs(np.median(lab) - lab).mean()
    n_plain = np.mean([r.nodes_expanded for r in plain])
    n_seed = np.mean([r.nodes_expanded for r in seeded])
    g_plain = ctx.estimate_batched(sen, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, gamma=0.025)
    g_seed = ctx.estimate_learned(net, sen, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps, gamma=0.025)
    ng_plain = sum(r.nodes_expanded for r in g_plain)
    ng_seed = sum(r.nodes_expanded for r in g_seed)
    print(f"network |d - d_hat| {err:.4f} (constant guess {const:.4f}); nodes per window "
          f"{n_plain:.2f} without seeds, {n_seed:.2f} with; gamma 0.025: {ng_plain} and {ng_seed} nodes")
    assert err < 0.05 and err < 0.25 * const
    assert n_seed < n_plain and ng_seed < ng_plain
    for r, q in zip(g_seed, plain):  # gamma-optimal
        assert q.contrast - r.contrast <= 0.025 + 1e-12
    dimgs = ctx.downsample(sen, x, y, off)  # bfloat16 bits on the device
    net.forward(dimgs)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(10):
        net.forward(dimgs)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - a) / 10
    a = time.perf_counter()
    for _ in range(3):
        ctx.estimate_learned(net, sen, x, y, t, off, tau, s.d_lo, s.d_hi, s.eps)
    torch.cuda.synchronize()
    t_search = (time.perf_counter() - a) / 3
    print(f"forward {t_fwd * 1e3:.3f} ms for {len(wins)} images, seeded search {t_search * 1e3:.2f} ms")
    assert t_fwd < 0.02 * t_search
    net.close()


def test_trained_1280x720_network_gains_on_the_benchmark_windows(ctx):
    """The committed network of the 1280x720 sensor (trained on windows from
    index 100000 on) on the benchmark's first 64 windows: its error against
    the certified optimum beats a constant guess; the optimum is the same
    with and without its seeds; the seeds save node expansions in the
    canonical search and with the gamma stop of Sec. 6."""
    import os

    import torch

    from paper_2209_13168_amd import ecmd, learned
    from paper_2209_13168_amd.learned import windows_chunks

    path = os.path.join(os.path.dirname(learned.__file__), "weights", "cnn_c5.npz")
    assert os.path.exists(path), "trained weights are missing"
    net, meta = learned.load(ctx, path)
    assert meta["config"] == "c5" and meta["first_window"] >= 1000
    x, y, t, off, tau, _ = next(windows_chunks(list(range(64)), cfg="c5", chunk=64))
    dev = torch.device("cuda:0")
    x, y, t, off, tau = (torch.from_numpy(a).to(dev) for a in (x, y, t, off, tau))
    _, _, _, sensor, search = learned.SETUPS["c5"]
    sen = ecmd.sensor(*sensor)
    plain = ctx.estimate_batched(sen, x, y, t, off, tau, **search)
    seeded = ctx.estimate_learned(net, sen, x, y, t, off, tau, **search)
    assert [(r.j_star, r.K) for r in plain] == [(r.j_star, r.K) for r in seeded]
    pred = net.forward(ctx.downsample(sen, x, y, off)).cpu().numpy()
    lab = np.array([r.d_hat for r in plain])
    err = np.abs(pred - lab).mean()
    const = np.abs(np.median(lab) - lab).mean()
    n_plain = sum(r.nodes_expanded for r in plain)
    n_seed = sum(r.nodes_expanded for r in seeded)
    g_plain = ctx.estimate_batched(sen, x, y, t, off, tau, **search, gamma=0.025)
    g_seed = ctx.estimate_learned(net, sen, x, y, t, off, tau, **search, gamma=0.025)
    ng_plain = sum(r.nodes_expanded for r in g_plain)
    ng_seed = sum(r.nodes_expanded for r in g_seed)
    print(f"network |d - d_hat| {err:.4f} (constant guess {const:.4f}); nodes {n_plain} without seeds, "
          f"{n_seed} with; gamma 0.025: {ng_plain} and {ng_seed}")
    assert err < 0.5 * const
    assert n_seed < n_plain and ng_seed < ng_plain
    M2 = float(sensor[0] * sensor[1]) ** 2
    for r, q in zip(g_seed, plain):  # gamma-optimal, with a gap that covers the loss
        assert 0.0 <= (q.K - r.K) / M2 <= r.gap + 1e-12 and r.gap <= 0.025
    net.close()
