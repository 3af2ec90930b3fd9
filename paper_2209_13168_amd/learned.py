"""Training and evaluation driver of the learned incumbent.

One network per sensor.  Data: windows of that sensor's generator, drawn on
the host cores -- for 346x260 the 100k-event generator with true D ~
U(0.05, 0.8); for 1280x720 the stress generator (0.1-5M events, 0.1% hot
pixels, D in [0, 2]) at window indices from TRAIN_BASE on, so that the
benchmark's windows 0-255 stay held out.  Each window's 64x64 input image
comes from the library's downsample kernel and its label is the certified
branch-and-bound optimum d_hat from the library (the network learns to
propose the BnB's own answer).  Training runs the library's
forward/backward/Adam kernels.

    python -m paper_2209_13168_amd.learned train --config c2 --windows 20000 \
        --out paper_2209_13168_amd/weights/cnn_c2.npz
    python -m paper_2209_13168_amd.learned train --config c5 --windows 6000 \
        --out paper_2209_13168_amd/weights/cnn_c5.npz
    python -m paper_2209_13168_amd.learned eval --config c5 --weights ... --eval-windows 256
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2209_13168_amd import ecmd  # noqa: E402

HELD_OUT = 1_000_000  # 346x260 generator: window indices from here on are never trained on
TRAIN_BASE = 100_000  # 1280x720: training windows start here (the benchmark uses 0-255)


def _gen(args):
    cfg, k, n_events = args
    from synth import config_windows

    kw = {"n_events": n_events} if n_events else {}
    w = config_windows(cfg, [k], **kw)[0]
    return w.x, w.y, w.t_rel, np.float32(w.spec.tau), w.spec.d_true


def windows_chunks(indices, cfg="c4", n_events=None, chunk=256, procs=None):
    """Yield (x, y, t_rel, offsets, tau, d_true) for consecutive chunks."""
    procs = procs or min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(procs) as ex:
        for c0 in range(0, len(indices), chunk):
            part = list(ex.map(_gen, [(cfg, int(k), n_events) for k in indices[c0:c0 + chunk]]))
            offs = np.zeros(len(part) + 1, np.int64)
            offs[1:] = np.cumsum([p[0].shape[0] for p in part])
            yield (np.concatenate([p[0] for p in part]), np.concatenate([p[1] for p in part]),
                   np.concatenate([p[2] for p in part]), offs, np.array([p[3] for p in part], np.float32),
                   np.array([p[4] for p in part]))


SEARCH = dict(d_lo=0.0, d_hi=1.5, eps=1e-5)
SENSOR = (346, 260, (173.0, 130.0))
# per sensor: (generator, first training window, first held-out window, sensor, search)
SETUPS = {
    "c2": ("c4", 0, HELD_OUT, SENSOR, SEARCH),
    "c5": ("c5", TRAIN_BASE, 0, (1280, 720, (640.0, 360.0)), dict(d_lo=0.0, d_hi=2.0, eps=1e-5)),
}


def label_chunk(ctx, x, y, t, offs, tau, device=True, seeds=None, net=None, setup="c2"):
    """Downsampled images (GPU) and certified optima (GPU BnB) of a chunk."""
    import torch

    _, _, _, sensor, search = SETUPS[setup]
    sen = ecmd.sensor(*sensor)
    if device:
        dev = torch.device("cuda:0")
        x, y, t, offs, tau = (torch.from_numpy(a).to(dev) for a in (x, y, t, offs, tau))
    imgs = ctx.downsample(sen, x, y, offs)
    if net is not None:
        res = ctx.estimate_learned(net, sen, x, y, t, offs, tau, **search)
    else:
        res = ctx.estimate_batched(sen, x, y, t, offs, tau, **search, d_seeds=seeds)
    if device:
        imgs = imgs.cpu().numpy().view(np.uint16)
    return imgs.reshape(-1, 64 * 64), res


def build_dataset(ctx, indices, n_events=None, log=print, setup="c2"):
    gen, base = SETUPS[setup][:2]
    imgs, labels, truth = [], [], []
    t0 = time.time()
    chunk = 256 if setup == "c2" else 64
    for x, y, t, offs, tau, dt in windows_chunks([base + int(k) for k in indices], cfg=gen, n_events=n_events,
                                                 chunk=chunk):
        im, res = label_chunk(ctx, x, y, t, offs, tau, setup=setup)
        imgs.append(im)
        labels.append(np.array([r.d_hat for r in res], np.float32))
        truth.append(dt)
        log(f"labelled {sum(len(a) for a in labels)} windows ({time.time() - t0:.0f} s)")
    return np.concatenate(imgs), np.concatenate(labels), np.concatenate(truth)


def train(ctx, imgs, labels, epochs=30, batch=256, lr=2e-3, seed=0, log=print):
    import torch

    dev = torch.device("cuda:0")
    X = torch.from_numpy(imgs.view(np.int16)).to(dev)
    Y = torch.from_numpy(labels).to(dev)
    net = ecmd.Cnn(ctx, seed=seed)
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        tot = 0.0
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tot += net.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr_ep)
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"epoch {ep}: mse {hist[-1]:.3e} (rmse {np.sqrt(hist[-1]):.4f})")
    return net, hist


def save(net, path, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.params(), meta=json.dumps(meta))


def load(ctx, path):
    z = np.load(path, allow_pickle=False)
    net = ecmd.Cnn(ctx, seed=0)
    net.set_params(z["params"])
    return net, json.loads(str(z["meta"]))


def evaluate(ctx, net, n_windows=256, n_events=None, log=print, setup="c2", label_mean=0.425):
    """Network error against the BnB optimum, and the search with and
    without the network's seeds on held-out windows (label_mean: the
    training labels' mean, the constant predictor compared against; 0.425
    is the mean of U(0.05, 0.8))."""
    gen, _, held = SETUPS[setup][:3]
    err, err_mean, plain_nodes, seeded_nodes, plain_steps, seeded_steps = [], [], [], [], [], []
    same = True
    chunk = 256 if setup == "c2" else 64
    for x, y, t, offs, tau, dt in windows_chunks(list(range(held, held + n_windows)), cfg=gen, n_events=n_events,
                                                 chunk=chunk):
        im, plain = label_chunk(ctx, x, y, t, offs, tau, setup=setup)
        _, seeded = label_chunk(ctx, x, y, t, offs, tau, net=net, setup=setup)
        pred = net.forward(im)
        lab = np.array([r.d_hat for r in plain])
        err.append(np.abs(pred - lab))
        err_mean.append(np.abs(label_mean - lab))
        plain_nodes += [r.nodes_expanded for r in plain]
        seeded_nodes += [r.nodes_expanded for r in seeded]
        plain_steps += [r.steps for r in plain]
        seeded_steps += [r.steps for r in seeded]
        same &= all((a.j_star, a.K) == (b.j_star, b.K) for a, b in zip(plain, seeded))
    err = np.concatenate(err)
    out = {
        "windows": int(err.size),
        "net_abs_err_mean": float(err.mean()),
        "net_abs_err_p90": float(np.percentile(err, 90)),
        "mean_predictor_abs_err": float(np.concatenate(err_mean).mean()),
        "nodes_plain_mean": float(np.mean(plain_nodes)),
        "nodes_seeded_mean": float(np.mean(seeded_nodes)),
        "steps_plain_mean": float(np.mean(plain_steps)),
        "steps_seeded_mean": float(np.mean(seeded_steps)),
        "same_optima": bool(same),
    }
    log(json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--config", choices=sorted(SETUPS), default="c2", help="sensor: c2 = 346x260, c5 = 1280x720")
    ap.add_argument("--windows", type=int, default=20000)
    ap.add_argument("--events", type=int, default=0, help="events per window (0 = the generator's)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--out", default=None, help="default: weights/cnn_<config>.npz")
    ap.add_argument("--weights", default=None, help="default: weights/cnn_<config>.npz")
    ap.add_argument("--eval-windows", type=int, default=256)
    a = ap.parse_args()
    path = os.path.join(os.path.dirname(__file__), "weights", f"cnn_{a.config}.npz")
    ctx = ecmd.Context(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if a.cmd == "train":
        imgs, labels, truth = build_dataset(ctx, range(a.windows), n_events=a.events or None, log=log,
                                            setup=a.config)
        log(f"label vs true D: mean abs {np.abs(labels - truth).mean():.4f}")
        net, hist = train(ctx, imgs, labels, epochs=a.epochs, log=log)
        meta = {"config": a.config, "generator": SETUPS[a.config][0], "first_window": SETUPS[a.config][1],
                "windows": int(a.windows), "events": a.events or "generator", "epochs": a.epochs,
                "final_train_mse": hist[-1], "labels": "certified BnB optimum d_hat",
                "label_mean": float(labels.mean())}
        out = a.out or path
        save(net, out, meta)
        meta["eval"] = evaluate(ctx, net, a.eval_windows, n_events=a.events or None, log=log, setup=a.config,
                                label_mean=float(labels.mean()))
        save(net, out, meta)
    else:
        net, meta = load(ctx, a.weights or path)
        evaluate(ctx, net, a.eval_windows, n_events=a.events or None, log=log, setup=a.config,
                 label_mean=float(meta.get("label_mean", 0.425)))


if __name__ == "__main__":
    main()
