"""Forward model of ventral descent onto a flat textured plane.

The scene model follows the geometry of the paper's Sec. 3 (eqs. (5)-(6)):
with the camera's vertical velocity constant over the window and depth
normalised to 1 at the window start, a surface point seen at image offset
``u(t)`` from the focus of expansion (FOE) moves radially as
``u(t) = u0 / (1 - D t)``, where ``D >= 0`` is the divergence magnitude at the
window start (the paper's ``-nu`` with ``Z0 = 1``).  Every signal event below
is a noisy sample of that trajectory, so the true divergence of a window is
known exactly.

Event recipe (one window):

* ``n_points`` surface points; point ``j`` ends the window at a position drawn
  uniformly on the sensor, so its whole trajectory stays on the sensor.
* signal events pick a point (equal rate, or "textured": rate proportional to
  ``Exp(1) * (0.25 + |u_end| / r_max)``), a time ``t ~ U[0, tau)``, and sit at
  the point's trajectory position plus optional Gaussian jitter (redrawn while
  off-sensor);
* noise events are uniform over the sensor and the window;
* hot pixels (optional) fire at a fixed rate with a random phase, at the
  pixel centre, on top of ``n_events``;
* polarity is +-1 uniform (the estimator ignores it);
* events are sorted by time.

Seeds: ``SeedSequence([2209, config_id, window_index, stream])``; stream 0
draws the window's parameters (event count, true D), stream 1 the events.
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "tiny", "noisefree")
_CONFIG_IDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "tiny": 90, "noisefree": 91}


@dataclass(frozen=True)
class WindowSpec:
    """Parameters of one synthetic window (all times in seconds)."""

    width: int
    height: int
    foe: Tuple[float, float]
    tau: float
    n_events: int  # signal + uniform noise; hot-pixel events come on top
    d_true: float
    n_points: int
    noise_frac: float
    jitter: float = 0.0  # px standard deviation per coordinate
    textured: bool = False
    hot_frac: float = 0.0  # fraction of pixels that are hot
    hot_rate_hz: float = 1000.0
    d_lo: float = 0.0  # search range of the estimator
    d_hi: float = 1.0
    eps: float = 1e-4
    t0: float = 100.0  # absolute start of the window


@dataclass
class Window:
    """One generated window. ``t`` is absolute (float64); ``t_rel`` is the
    float32 offset from ``spec.t0`` and ``t == t0 + float64(t_rel)`` holds
    exactly, so ``float32(t - t0) == t_rel``."""

    spec: WindowSpec
    x: np.ndarray  # float32 [N]
    y: np.ndarray  # float32 [N]
    t_rel: np.ndarray  # float32 [N], in [0, tau)
    p: np.ndarray  # int8 [N]
    owner: np.ndarray  # int32 [N]: source surface point of a signal event, -1 otherwise
    n_signal: int
    n_noise: int
    n_hot: int

    @property
    def t(self) -> np.ndarray:
        return np.float64(self.spec.t0) + self.t_rel.astype(np.float64)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def t1(self) -> float:
        return float(self.spec.t0) + float(np.float32(self.spec.tau))


def _rng(cfg_id: int, k: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2209, cfg_id, k, stream])))


def _f32_below(v: np.ndarray, hi: float) -> np.ndarray:
    """float32 of ``v`` with values that round up to ``hi`` pulled just below."""
    out = v.astype(np.float32)
    top = np.nextafter(np.float32(hi), np.float32(0))
    return np.minimum(out, top)


def make_window(spec: WindowSpec, cfg_id: int, k: int) -> Window:
    rng = _rng(cfg_id, k, 1)
    W, H = spec.width, spec.height
    cx, cy = spec.foe
    tau32 = np.float32(spec.tau)
    n_noise = int(round(spec.n_events * spec.noise_frac))
    n_signal = spec.n_events - n_noise

    # surface points: end-of-window positions uniform on the sensor
    pe_x = rng.uniform(0.0, W, spec.n_points)
    pe_y = rng.uniform(0.0, H, spec.n_points)
    if spec.textured:
        r_max = max(math.hypot(cx - a, cy - b) for a in (0.0, W) for b in (0.0, H))
        w = rng.exponential(1.0, spec.n_points) * (0.25 + np.hypot(pe_x - cx, pe_y - cy) / r_max)
        owner = rng.choice(spec.n_points, size=n_signal, p=w / w.sum())
    else:
        owner = rng.permutation(np.arange(n_signal) % max(spec.n_points, 1))

    def draw_times(n: int) -> np.ndarray:
        t = rng.uniform(0.0, float(tau32), n).astype(np.float32)
        return np.minimum(t, np.nextafter(tau32, np.float32(0)))

    # signal events on the radial trajectories u(t) = u0 / (1 - D t)
    ts = draw_times(n_signal)
    D = spec.d_true
    scale0 = 1.0 - D * float(tau32)
    u0x = (pe_x[owner] - cx) * scale0
    u0y = (pe_y[owner] - cy) * scale0
    g = 1.0 / (1.0 - D * ts.astype(np.float64))
    sx = cx + u0x * g
    sy = cy + u0y * g
    if spec.jitter > 0.0:
        jx = sx + rng.normal(0.0, spec.jitter, n_signal)
        jy = sy + rng.normal(0.0, spec.jitter, n_signal)
        for _ in range(1000):
            bad = (jx < 0) | (jx >= W) | (jy < 0) | (jy >= H)
            nb = int(bad.sum())
            if nb == 0:
                break
            jx[bad] = sx[bad] + rng.normal(0.0, spec.jitter, nb)
            jy[bad] = sy[bad] + rng.normal(0.0, spec.jitter, nb)
        else:  # pragma: no cover - practically unreachable
            jx, jy = np.clip(jx, 0, W), np.clip(jy, 0, H)
        sx, sy = jx, jy

    # uniform noise
    nx = rng.uniform(0.0, W, n_noise)
    ny = rng.uniform(0.0, H, n_noise)
    tn = draw_times(n_noise)

    # hot pixels at pixel centres
    hx = np.zeros(0)
    hy = np.zeros(0)
    th = np.zeros(0, np.float32)
    n_hotpix = int(round(spec.hot_frac * W * H))
    if n_hotpix > 0:
        pix = rng.choice(W * H, size=n_hotpix, replace=False)
        period = 1.0 / spec.hot_rate_hz
        phase = rng.uniform(0.0, period, n_hotpix)
        counts = np.floor((float(tau32) - phase) / period).astype(np.int64) + 1
        counts = np.maximum(counts, 0)
        rep = np.repeat(np.arange(n_hotpix), counts)
        kk = np.arange(rep.size) - np.repeat(np.cumsum(counts) - counts, counts)
        th = (phase[rep] + kk * period).astype(np.float32)
        keep = th < tau32
        rep, th = rep[keep], th[keep]
        hx = (pix[rep] % W) + 0.5
        hy = (pix[rep] // W) + 0.5

    x = _f32_below(np.concatenate([sx, nx, hx]), W)
    y = _f32_below(np.concatenate([sy, ny, hy]), H)
    t = np.concatenate([ts, tn, th]).astype(np.float32)
    p = rng.choice(np.array([-1, 1], np.int8), size=x.size)
    own = np.concatenate([owner.astype(np.int32), np.full(n_noise + hx.size, -1, np.int32)])
    order = np.argsort(t, kind="stable")
    return Window(spec=spec, x=x[order], y=y[order], t_rel=t[order], p=p[order],
                  owner=own[order], n_signal=n_signal, n_noise=n_noise, n_hot=int(hx.size))


def config_specs(name: str, k: int) -> WindowSpec:
    """The spec of window ``k`` of a named configuration."""
    cid = _CONFIG_IDS[name]
    rng = _rng(cid, k, 0)
    if name == "c1":
        return WindowSpec(128, 128, (64.0, 64.0), 0.5, 10_000, 0.3, 300, 0.10,
                          d_lo=0.0, d_hi=1.0, eps=1e-4)
    if name == "noisefree":
        return WindowSpec(128, 128, (64.0, 64.0), 0.5, 10_000, 0.3, 300, 0.0,
                          d_lo=0.0, d_hi=1.0, eps=1e-4)
    if name in ("c2", "c4"):
        D = float(rng.uniform(0.05, 0.8))
        return WindowSpec(346, 260, (173.0, 130.0), 0.25, 100_000, D, 2000, 0.20,
                          jitter=0.5, textured=True, d_lo=0.0, d_hi=1.5, eps=1e-5)
    if name == "c3":
        n = int(round(math.exp(rng.uniform(math.log(5e4), math.log(1e6)))))
        D = 0.1 + 0.5 * (k % 64) / 63.0
        return WindowSpec(640, 480, (320.0, 240.0), 0.25, n, D, 6830, 0.20,
                          jitter=0.5, textured=True, d_lo=0.0, d_hi=1.5, eps=1e-5)
    if name == "c5":
        n = int(round(math.exp(rng.uniform(math.log(1e5), math.log(5e6)))))
        D = float(rng.uniform(0.05, 1.5))
        return WindowSpec(1280, 720, (640.0, 360.0), 0.25, n, D, 20490, 0.30,
                          jitter=0.5, textured=True, hot_frac=0.001, hot_rate_hz=1000.0,
                          d_lo=0.0, d_hi=2.0, eps=1e-5)
    if name == "tiny":
        n = int(rng.integers(8, 65))
        D = float(rng.uniform(0.1, 1.2))
        return WindowSpec(16, 16, (8.0, 8.0), 0.5, n, D, max(1, n // 6), 0.25,
                          jitter=0.0, d_lo=0.0, d_hi=1.5, eps=1e-3)
    raise KeyError(name)


def config_windows(name: str, indices: Sequence[int], **overrides) -> List[Window]:
    """Generate windows ``indices`` of configuration ``name``.

    ``overrides`` replace spec fields (e.g. ``n_events=20_000`` for a smaller
    test window of the same shape)."""
    cid = _CONFIG_IDS[name]
    out = []
    for k in indices:
        spec = config_specs(name, k)
        if overrides:
            spec = dataclasses.replace(spec, **overrides)
        out.append(make_window(spec, cid, k))
    return out


def pack_batch(windows: Sequence[Window]):
    """Concatenate windows into the CSR layout of the batched entry point:
    ``(x, y, t_rel, offsets[B+1] int64, tau[B] float32)``."""
    offs = np.zeros(len(windows) + 1, np.int64)
    offs[1:] = np.cumsum([w.n for w in windows])
    x = np.concatenate([w.x for w in windows]) if windows else np.zeros(0, np.float32)
    y = np.concatenate([w.y for w in windows]) if windows else np.zeros(0, np.float32)
    t = np.concatenate([w.t_rel for w in windows]) if windows else np.zeros(0, np.float32)
    tau = np.array([np.float32(w.spec.tau) for w in windows], np.float32)
    return x, y, t, offs, tau
