"""Continuum optimum of the contrast over d for tiny inputs (fp64).

TEST INFRASTRUCTURE ONLY.  With the warp of eq. (12) evaluated exactly, the
event image H(u; d) only changes where some warped coordinate crosses an
integer (a pixel edge, including the image border).  Between two consecutive
such breakpoints the contrast of eq. (14) is constant, so evaluating it once
inside every elementary interval gives the exact maximum over the continuum.

Breakpoints: x + ax*r = k  =>  r = (k - x)/ax, and d = r/(1 + r*tau) inverts
r = d/(1 - d*tau).  Meant for a few dozen events on a small sensor.
"""

from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def breakpoints(ev: "O.Events", d_lo: float, d_hi: float) -> np.ndarray:
    tau = float(ev.tau)
    x = ev.x.astype(np.float64)
    y = ev.y.astype(np.float64)
    delta = tau - ev.t.astype(np.float64)
    ax = (x - float(ev.cx)) * delta
    ay = (y - float(ev.cy)) * delta
    r_lo = d_lo / (1.0 - d_lo * tau)
    r_hi = d_hi / (1.0 - d_hi * tau)
    rs = []
    for p, a, lim in ((x, ax, ev.W), (y, ay, ev.H)):
        for i in range(p.shape[0]):
            if a[i] == 0.0:
                continue
            lo = p[i] + a[i] * r_lo
            hi = p[i] + a[i] * r_hi
            k0, k1 = math.floor(min(lo, hi)), math.ceil(max(lo, hi))
            for k in range(max(k0, 0), min(k1, lim) + 1):
                r = (k - p[i]) / a[i]
                if r_lo < r < r_hi:
                    rs.append(r)
    r = np.unique(np.array(rs, np.float64))
    d = r / (1.0 + r * tau)
    return np.concatenate([[d_lo], d, [d_hi]])


def continuum_max(ev: "O.Events", d_lo: float, d_hi: float):
    """Return (C_max, bp, C_mid): the maximum contrast over [d_lo, d_hi], the
    sorted breakpoints and the contrast inside each elementary interval."""
    bp = breakpoints(ev, d_lo, d_hi)
    mids = 0.5 * (bp[:-1] + bp[1:])
    M = ev.M
    C_mid = np.empty(mids.shape[0])
    for i, d in enumerate(mids):
        S, N = O.point64(ev, float(d))
        C_mid[i] = O.key(M, S, N) / float(M) / float(M)
    return float(C_mid.max()), bp, C_mid
