"""The pins catch plausible mistakes: each case plants one mistake in a copy
of the oracle's C source (on the CPU only), builds it, and checks that at
least one pin of ``test_oracle_pins`` fails against it."""

import os
import subprocess

import pytest

from tests import test_oracle_pins as P

MUTANTS = {
    # transposed pixel index (x and y swapped in the flat index)
    "pixel_index_transposed": [("pix[i] = ky * W + kx;", "pix[i] = kx * H + ky;"),
                               ("img[(int64_t)ky * W + kx] += 1;", "img[(int64_t)kx * H + ky] += 1;")],
    # wrong sign of the divergence in the denominator of eq. (12)
    "denominator_sign": [("float den = 1.0f - a;", "float den = 1.0f + a;")],
    # elapsed time instead of time to the window end
    "delta_uses_t": [("float delta = tau - t_rel[i];", "float delta = t_rel[i];")],
    # the mean term of eq. (14) dropped from the key
    "key_drops_mean": [("return (i128)M * (i128)S - (i128)N * (i128)N;", "return (i128)M * (i128)S;")],
    # walk decides corners the wrong way round
    "walk_corner_swapped": [("double e = ex - ey;", "double e = ey - ex;")],
    # eq. (20) read as "touches the image" instead of "fully inside"
    "mu_low_any_endpoint": [("if (inside32(xa, ya, W, H) && inside32(xb, yb, W, H)) n_low += 1;",
                             "if (inside32(xa, ya, W, H) || inside32(xb, yb, W, H)) n_low += 1;")],
    # walk forgets the both-sides case at near corners
    "walk_no_corner_slack": [("double thr = ldexp(fabs(ax) + fabs(ay), -8);", "double thr = 0.0;")],
    # incumbent tie broken towards the larger index
    "tie_prefers_larger_j": [("(Kc == K_inc && jc < j_inc)", "(Kc == K_inc && jc > j_inc)")],
    # children of 4-wide nodes never split
    "split_off_by_one": [("if (nd.jb - nd.ja >= 4) {", "if (nd.jb - nd.ja > 4) {")],
}

PINS = [
    lambda o: P.test_pixels_match_independent_numpy_warp(o, "c2", 20_000),
    lambda o: P.test_point_value_is_bincount_and_variance(o, "c1", None),
    lambda o: P.test_key_closed_forms(o),
    lambda o: P.test_signal_events_collapse_at_true_divergence(o),
    lambda o: P.test_bound_equals_point_at_singletons(o),
    lambda o: P.test_bound_dominates_every_fp32_point(o, "c2", None),
    lambda o: P.test_bound_many_random_points_c1(o),
    lambda o: P.test_walk_is_thin_single_events(o),
    lambda o: P.test_bound_valid_near_pixel_corners(o),
    lambda o: [P.test_bnb_equals_dense_sweep_tiny(o, k) for k in range(12)],
    lambda o: P.test_bnb_equals_dense_sweep_c1(o),
    lambda o: P.test_recovers_true_divergence_noise_free(o),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(orc, tmp_path, name):
    src = open(orc.SRC).read()
    for old, new in MUTANTS[name]:
        assert old in src, (name, old)
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(src)
    so = str(tmp_path / "libmutant.so")
    subprocess.run(["cc", *orc.CFLAGS, str(c), "-o", so, "-lm"], check=True)
    caught = []
    with orc.using(so):
        for pin in PINS:
            try:
                pin(orc)
            except AssertionError:
                caught.append(pin)
                break
    assert caught, f"no pin fails with the planted mistake {name}"
    assert os.path.exists(orc.LIB)
