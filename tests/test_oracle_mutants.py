"""The pins catch plausible mistakes: each case plants one mistake in a copy
of the oracle's C source (on the CPU only), builds it, and checks that at
least one pin of ``test_oracle_pins`` fails against it."""

import os
import subprocess

import pytest

from tests import test_oracle_pins as P
from tests import test_oracle_polarity as PP

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

# planted mistakes in the polarity-aware statement, caught by its own pins
POL_MUTANTS = {
    # the key counts the cells of one image only
    "pol_key_uses_M": [("return key_of(2 * k->M, S, N);", "return key_of(k->M, S, N);"),
                       ("return key_of(2 * k->M, S, n_low);", "return key_of(k->M, S, n_low);"),
                       ("rc = bnb_run(&k, ptpol, bdpol, L, 2 * k.M,", "rc = bnb_run(&k, ptpol, bdpol, L, k.M,")],
    # both polarities binned into the same image
    "pol_same_image": [("point_image32(s.e[1], s.n[1], W, H, r, img + M);",
                        "point_image32(s.e[1], s.n[1], W, H, r, img);"),
                       ("point_image32(k->s.e[1], k->s.n[1], k->W, k->H, k->r[j], k->img + k->M);",
                        "point_image32(k->s.e[1], k->s.n[1], k->W, k->H, k->r[j], k->img);")],
    # zero polarity counted as positive (split on >= 0)
    "pol_split_sign": [("for (int64_t i = 0; i < n; ++i) m += ((pol[i] > 0) == l);",
                        "for (int64_t i = 0; i < n; ++i) m += ((pol[i] >= 0) == l);"),
                       ("if ((pol[i] > 0) != l) continue;", "if ((pol[i] >= 0) != l) continue;")],
    # N_low of the second image dropped from the bound
    "pol_bound_drops_nlow": [("int64_t n_low = bound_image32(k->s.e[0], k->s.n[0], k->W, k->H, k->r[ja], k->r[jb], k->img)\n"
                              "                  + bound_image32(",
                              "int64_t n_low = bound_image32(k->s.e[0], k->s.n[0], k->W, k->H, k->r[ja], k->r[jb], k->img);\n"
                              "    (void)bound_image32(")],
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


POL_PINS = [
    lambda o: PP.test_point_pol_is_bincount_over_two_images(o, "c1", None),
    lambda o: PP.test_doubled_window_closed_form(o),
    lambda o: PP.test_bound_pol_dominates_points(o),
    lambda o: [PP.test_bnb_pol_equals_brute_force_tiny(o, k) for k in range(8)],
    lambda o: PP.test_polarity_flip_and_single_polarity(o),
]


@pytest.mark.parametrize("name", sorted(POL_MUTANTS))
def test_polarity_pins_catch_planted_mistake(orc, tmp_path, name):
    src = open(orc.SRC).read()
    for old, new in POL_MUTANTS[name]:
        assert old in src, (name, old)
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(src)
    so = str(tmp_path / "libmutant.so")
    subprocess.run(["cc", *orc.CFLAGS, str(c), "-o", so, "-lm"], check=True)
    caught = []
    with orc.using(so):
        for pin in POL_PINS:
            try:
                pin(orc)
            except AssertionError:
                caught.append(pin)
                break
    assert caught, f"no polarity pin fails with the planted mistake {name}"
