"""CPU statement of the event preprocessing of Sec. 6 (NumPy).

TEST INFRASTRUCTURE ONLY.
  hot_pixel_filter: drop every event of a pixel (floor(x), floor(y)) holding
      more than max_count events of its window;
  resample: scale coordinates by float32(W_out / W_in), float32(H_out / H_in)
      and keep event k of window w iff the top 24 bits of SplitMix64 at
      seed + (w * 2^32 + k + 1) * 0x9E3779B97F4A7C15 are below
      floor(keep_frac * 2^24).  SplitMix64 (Steele, Lea, Flood 2014): add the
      golden-ratio increment, then z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
      z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31 (mod 2^64).
Both keep the order of the events and return (x, y, t, offsets).
"""

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _compact(x, y, t, offsets, keep, sx=np.float32(1), sy=np.float32(1)):
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    t = np.asarray(t, np.float32)
    o = np.asarray(offsets, np.int64)
    idx = np.arange(o[0], o[-1])
    kept = idx[keep]
    new_off = np.concatenate([[0], np.cumsum([int(keep[o[w] - o[0]:o[w + 1] - o[0]].sum()) for w in range(len(o) - 1)])])
    return (x[kept] * np.float32(sx)).astype(np.float32), (y[kept] * np.float32(sy)).astype(np.float32), \
        t[kept], new_off.astype(np.int64)


def hot_pixel_filter(x, y, t, offsets, W, H, max_count):
    o = np.asarray(offsets, np.int64)
    keep = np.ones(o[-1] - o[0], bool)
    for w in range(len(o) - 1):
        a, b = o[w], o[w + 1]
        xs = np.asarray(x[a:b], np.float32)
        ys = np.asarray(y[a:b], np.float32)
        ins = (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
        pix = np.floor(ys).astype(np.int64) * W + np.floor(xs).astype(np.int64)
        cnt = np.bincount(pix[ins], minlength=W * H)
        k = np.ones(b - a, bool)
        k[ins] = cnt[pix[ins]] <= max_count
        keep[a - o[0]:b - o[0]] = k
    return _compact(x, y, t, o, keep)


def resample_keep(offsets, keep_frac, seed):
    o = np.asarray(offsets, np.int64)
    th = np.uint64(int(np.floor(np.float64(np.float32(keep_frac)) * 16777216.0)))
    keep = np.empty(o[-1] - o[0], bool)
    for w in range(len(o) - 1):
        k = np.arange(o[w + 1] - o[w], dtype=np.uint64)
        ctr = (np.uint64(w) << np.uint64(32)) + k + np.uint64(1)
        with np.errstate(over="ignore"):
            z = _mix(np.uint64(seed) + ctr * GOLDEN)
        keep[o[w] - o[0]:o[w + 1] - o[0]] = (z >> np.uint64(40)) < th
    return keep


def resample(x, y, t, offsets, W_in, H_in, W_out, H_out, keep_frac, seed):
    keep = resample_keep(offsets, keep_frac, seed)
    sx = np.float32(W_out) / np.float32(W_in)
    sy = np.float32(H_out) / np.float32(H_in)
    return _compact(x, y, t, offsets, keep, sx, sy)
