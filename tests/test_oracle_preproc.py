"""Pins of the preprocessing statement: SplitMix64 against its published
first outputs, the keep rate, and the hot-pixel filter on a hand-made case."""

import numpy as np

from oracle import preproc


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 1234567: the first outputs of the published
    # generator (state += golden ratio, then the mix)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    s = np.uint64(1234567)
    got = []
    for k in range(1, 6):
        with np.errstate(over="ignore"):
            got.append(int(preproc._mix(np.array([s + np.uint64(k) * preproc.GOLDEN]))[0]))
    assert got == want


def test_resample_keep_rate_and_order():
    off = np.array([0, 40000, 40000, 100000], np.int64)
    keep = preproc.resample_keep(off, 0.25, 7)
    assert abs(keep.mean() - 0.25) < 0.01
    assert preproc.resample_keep(off, 1.0, 7).all() and not preproc.resample_keep(off, 0.0, 7).any()
    x = np.arange(100000, dtype=np.float32) % 346
    t = np.arange(100000, dtype=np.float32)
    xo, yo, to, oo = preproc.resample(x, x, t, off, 346, 260, 160, 90, 0.25, 7)
    assert oo[-1] == keep.sum() and list(oo[1:3]) == [keep[:40000].sum()] * 2
    assert np.all(np.diff(to) > 0)  # order kept
    assert xo.dtype == np.float32 and np.all(xo <= np.float32(160))


def test_hot_pixel_filter_hand_case():
    # window 0: pixel (2, 3) holds 5 events, pixel (7, 1) holds 2; window 1: pixel (2, 3) holds 1
    x = np.array([2.1, 2.9, 7.5, 2.5, 2.2, 7.1, 2.7, 2.0, 9.5], np.float32)
    y = np.array([3.5, 3.1, 1.2, 3.9, 3.0, 1.8, 3.3, 3.5, 9.9], np.float32)
    t = np.arange(9, dtype=np.float32)
    off = np.array([0, 7, 9], np.int64)
    xo, yo, to, oo = preproc.hot_pixel_filter(x, y, t, off, 10, 10, 3)
    assert list(to) == [2.0, 5.0, 7.0, 8.0] and list(oo) == [0, 2, 4]
