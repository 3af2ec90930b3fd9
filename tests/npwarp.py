"""Independent NumPy statement of the fp32 warp (used to pin the oracle).

Written from eq. (12) and the fp32 operation order the method fixes; shares
no code with the C oracle or the HIP path.  NumPy has no fp32 fused
multiply-add, so fmaf(a, r, x) is emulated: the product of two fp32 values is
exact in fp64, the fp64 sum rounds once and the cast to fp32 rounds again.
The second rounding can differ from a single correct rounding only when the
fp64 sum lands exactly on an fp32 midpoint; those elements are redone with
exact rational arithmetic.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

f32 = np.float32
f64 = np.float64


def _round_fraction_to_f32(v: Fraction, a: np.float32, b: np.float32) -> np.float32:
    """Correctly round the exact value v, known to lie between the adjacent
    fp32 values a and b, to nearest (ties to even)."""
    da = abs(v - Fraction(float(a)))
    db = abs(v - Fraction(float(b)))
    if da < db:
        return a
    if db < da:
        return b
    ia = np.array([a], f32).view(np.uint32)[0]
    return a if (ia & 1) == 0 else b


def fmaf(a: np.ndarray, r: np.float32, x: np.ndarray) -> np.ndarray:
    a = np.asarray(a, f32)
    x = np.asarray(x, f32)
    prod = a.astype(f64) * f64(r)  # exact: 24 + 24 bits
    s = prod + x.astype(f64)
    out = s.astype(f32)
    other = np.nextafter(out, np.where(s > out.astype(f64), f32(np.inf), f32(-np.inf)))
    mid = 0.5 * (out.astype(f64) + other.astype(f64))
    amb = (s != out.astype(f64)) & (s == mid)
    for i in np.nonzero(amb)[0]:
        v = Fraction(float(a[i])) * Fraction(float(r)) + Fraction(float(x[i]))
        out[i] = _round_fraction_to_f32(v, out[i], other[i])
    return out


def rate(d: float, tau: float) -> np.float32:
    d = f32(d)
    a = d * f32(tau)
    den = f32(1.0) - a
    return d / den


def warp(x, y, t_rel, tau, cx, cy, d):
    x = np.asarray(x, f32)
    y = np.asarray(y, f32)
    t = np.asarray(t_rel, f32)
    ux = x - f32(cx)
    uy = y - f32(cy)
    delta = f32(tau) - t
    ax = ux * delta
    ay = uy * delta
    r = rate(d, tau)
    return fmaf(ax, r, x), fmaf(ay, r, y)


def pixels(x, y, t_rel, tau, W, H, cx, cy, d) -> np.ndarray:
    xw, yw = warp(x, y, t_rel, tau, cx, cy, d)
    ins = (xw >= 0) & (xw < f32(W)) & (yw >= 0) & (yw < f32(H))
    kx = np.floor(xw).astype(np.int64)
    ky = np.floor(yw).astype(np.int64)
    return np.where(ins, ky * W + kx, -1).astype(np.int64)
