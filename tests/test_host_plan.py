"""Host logic of the library that needs no device: the grid (depth and grid
points) against the oracle's own statement of it, and the image tiling of
the evaluation kernel against its invariants (cuts at an integer FOE, tiles
within the LDS budget, segments within the kernel's limit)."""

import numpy as np
import pytest

from paper_2209_13168_amd import ecmd


def test_grid_depth_matches_the_oracle(orc):
    rng = np.random.default_rng(3)
    cases = [(0.0, 1.0, 1e-4), (0.0, 1.5, 1e-5), (0.0, 2.0, 1e-5), (0.0, 1.0, 0.25), (0.0, 1.0, 0.5),
             (0.2, 0.7, 2.0 ** -10), (0.0, 1.0, 2.0 ** -30)]
    for _ in range(200):
        lo = float(np.float32(rng.uniform(0, 1)))
        hi = float(np.float32(lo + rng.uniform(1e-3, 2)))
        cases.append((lo, hi, float(np.float32(10 ** rng.uniform(-8, 0)))))
    sen = ecmd.sensor(64, 48, (32, 24))
    for lo, hi, eps in cases:
        L = orc.depth(lo, hi, eps)
        if L < 1 or L > 30:
            continue
        assert ecmd.plan(sen, lo, hi, eps)["L"] == L, (lo, hi, eps)


def test_grid_points_match_the_oracle_bit_for_bit(orc):
    rng = np.random.default_rng(4)
    for _ in range(300):
        lo = float(np.float32(rng.uniform(0, 1)))
        hi = float(np.float32(lo + rng.uniform(1e-3, 2)))
        L = int(rng.integers(1, 31))
        for j in (0, 1, (1 << L) - 1, 1 << L, int(rng.integers(0, (1 << L) + 1))):
            a = np.float32(ecmd.grid_point(lo, hi, L, j))
            b = np.float32(orc.grid_d(lo, hi, L, j))
            assert a.view(np.uint32) == b.view(np.uint32), (lo, hi, L, j)
    assert np.isnan(ecmd.grid_point(0.0, 1.0, 0, 0)) and np.isnan(ecmd.grid_point(0.0, 1.0, 4, 17))


SENSORS = [(128, 128, (64, 64)), (346, 260, (173, 130)), (640, 480, (320, 240)), (1280, 720, (640, 360)),
           (346, 260, (101.3, 57.85)), (300, 200, (-5.0, 40.0)), (17, 5, (8, 2)), (1, 1, (0.5, 0.5)),
           (4096, 3000, (2048, 1500))]


@pytest.mark.parametrize("W,H,foe", SENSORS)
@pytest.mark.parametrize("pol", [False, True])
@pytest.mark.parametrize("tile_px", [0, 5000])
def test_tile_plan_invariants(W, H, foe, pol, tile_px):
    sen = ecmd.sensor(W, H, foe)
    try:
        p = ecmd.plan(sen, 0.0, 1.5, 1e-5, polarity=pol, tile_px=tile_px)
    except ecmd.EcmdError:
        # only a sensor that needs more tiles than the kernel holds may fail:
        # with at most 64 segments some tile has area A >= W*H/tiles, and its
        # counters (w + 2)(h + 2) >= A + 4 sqrt(A) + 4 exceed the budget
        A = W * H / (64 // (2 if pol else 1))
        budget = tile_px or 40_860
        assert A + 4 * np.sqrt(A) + 4 > budget
        return
    cc, rc = p["colcut"], p["rowcut"]
    assert cc[0] == 0 and cc[-1] == W and all(a < b for a, b in zip(cc, cc[1:]))
    assert rc[0] == 0 and rc[-1] == H and all(a < b for a, b in zip(rc, rc[1:]))
    # the FOE lines are cuts when the FOE is an integer point strictly inside
    for v, cuts, n in ((foe[0], cc, W), (foe[1], rc, H)):
        if float(v).is_integer() and 0 < v < n:
            assert int(v) in cuts
    widths, heights = np.diff(cc), np.diff(rc)
    assert p["max_tile_px"] == int(widths.max() * heights.max())
    # the counters of the largest tile, its one-cell border included, fit the budget
    assert int((widths.max() + 2) * (heights.max() + 2)) <= p["tile_budget_px"]
    if tile_px:
        assert p["tile_budget_px"] <= tile_px
    assert p["segments"] == p["ntx"] * p["nty"] * (2 if pol else 1) <= 64


def test_tile_counts_of_the_synthetic_sensors():
    """Default rule (160 KiB of LDS): tiles for three 512-thread workgroups per
    CU when that needs at most 24 tiles (quadrants halved on 346x260, 6 tiles
    per quadrant on 640x480), else for two, else the whole LDS for one
    1024-thread workgroup (1280x720: 24 tiles)."""
    want = {(128, 128): (4, 512), (346, 260): (8, 512), (640, 480): (24, 512), (1280, 720): (24, 1024)}
    for W, H, foe in SENSORS[:4]:
        p = ecmd.plan(ecmd.sensor(W, H, foe), 0.0, 1.5, 1e-5)
        q = ecmd.plan(ecmd.sensor(W, H, foe), 0.0, 1.5, 1e-5, polarity=True)
        assert (p["segments"], p["eval_threads"]) == want[(W, H)], (W, H, p)
        assert q["segments"] == 2 * p["segments"] and q["colcut"] == p["colcut"], (W, H, q)
        for r in (p, q):  # the workgroups' LDS fit the CU: three of 512 threads, or one of 1024
            k = 3 if r["eval_threads"] == 512 else 1
            assert k * (4 * r["tile_budget_px"] + 420) <= 160 * 1024


def test_plan_rejects_bad_arguments():
    with pytest.raises(ecmd.EcmdError):
        ecmd.plan(ecmd.sensor(0, 10, (0, 0)), 0.0, 1.0, 1e-3)
    with pytest.raises(ecmd.EcmdError):
        ecmd.plan(ecmd.sensor(10, 10, (5, 5)), 1.0, 0.5, 1e-3)
    with pytest.raises(ecmd.EcmdError):
        ecmd.plan(ecmd.sensor(10, 10, (5, 5)), 0.0, 1.0, 0.0)
