"""The pins must notice plausible mistakes: each test here plants one mistake in a
copy of the oracle source (on the CPU), rebuilds it, and requires at least one
pin to fail against it."""
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as pins
from tests import test_oracle_diode as dpins
from tests import test_oracle_sky as spins
from tests import test_oracle_trackers as tpins
from tests import test_oracle_depth_origin as zpins

SRC = open(O.SRC).read()

MUTANTS = {
    "fill_rule_flipped": ("topleft[e] = (dy < 0) || (dy == 0 && dx < 0);",
                          "topleft[e] = (dy > 0) || (dy == 0 && dx > 0);"),
    "pixel_centre_offset": ("int64_t px = i * 256 + 128;", "int64_t px = i * 256;"),
    "anchor_uses_wrong_gradient": ("za = (Z[0] + gx * (((double)i0 + 0.5)", "za = (Z[0] + gy * (((double)i0 + 0.5)"),
    "depth_fraction_bits": ("(j - j0) * gyf, 16);", "(j - j0) * gyf, 15);"),
    "farthest_depth_wins": ("if ((uint32_t)D < map[j * (int64_t)n + i])", "if ((uint32_t)D > map[j * (int64_t)n + i] || map[j * (int64_t)n + i] == OR_DMAX)"),
    "constant_bias_only": ("double b = ceil((0.5 + 1.0 / 512.0) * (gxs + gys)) + 2.0;", "double b = 2.0;"),
    "shade_test_reversed": ("int shaded = zs > ", "int shaded = zs < "),
    "sample_index_mixup": ("double fu = ((double)(k * cu + a) + 0.5)", "double fu = ((double)(k * cu + b) + 0.5)"),
    "view_toward_sun": ("V->d = mk(-s.x, -s.y, -s.z);", "V->d = mk(s.x, s.y, s.z);"),
    "window_without_margin": ("V->itx = (double)(n - 2) / su;", "V->itx = (double)(n) / su;"),
    "clip_midpoint": ("out[m][k] = p[k] + (r[k] - p[k]) * t;", "out[m][k] = p[k] + (r[k] - p[k]) * 0.5;"),
    "string_count_off_by_one": ("double p = (double)(j + 1) * caps[j];", "double p = (double)(j) * caps[j];"),
    "diffuse_dropped": ("double g = beam[m] * (1.0 - f) + d_poa * sky;", "double g = beam[m] * (1.0 - f);"),
    "back_lit_tested": ("if (!(cm > 0.0) || !V.valid) continue;\n        double nx = dot3(nh, V.e1), ny = dot3(nh, V.e2), nz = dot3(nh, V.d);\n        double gxs",
                        "if (!V.valid) continue;\n        double nx = dot3(nh, V.e1), ny = dot3(nh, V.e2), nz = dot3(nh, V.d);\n        double gxs"),
    "far_cull_inverted": ("if (zmin > (double)OR_DMAX) return;", "if (zmin < (double)OR_DMAX) return;"),
    "tracker_frame_mirrored": ("*v = cross3(*n, *u);", "*v = cross3(*u, *n);"),
    "one_axis_normal_not_projected": ("v3 q = mk(s.x - sa * T->a.x, s.y - sa * T->a.y, s.z - sa * T->a.z);",
                                      "v3 q = s;"),
    "pose_drops_height_over_pivot": ("o = add3(T->p, in_frame(dot3(r, u0), dot3(r, v0), dot3(r, n0), u, v, n));",
                                     "o = add3(T->p, in_frame(dot3(r, u0), dot3(r, v0), 0.0, u, v, n));"),
    "pose_edges_left_at_rest": ("U = in_frame(dot3(U, u0), dot3(U, v0), dot3(U, n0), u, v, n);", ""),
    "tracked_sphere_ignores_reach": ("OR_GROW(mk(trk[t].p.x + r, trk[t].p.y + r, trk[t].p.z + r));", ""),
    "diode_series_resistance_sign": ("return x - I * d[4];", "return x + I * d[4];"),
    "diode_shunt_dropped": ("double f = (c - d[2] * e) - x / d[5];", "double f = c - d[2] * e;"),
    "diode_photocurrent_unscaled": ("double iph = d[0] * G / d[1];", "double iph = d[0];"),
    "bypass_diode_missing": ("if (vs < -d[6]) vs = -d[6];", ""),
    "mpp_not_refined": ("for (int it = 0; it < OR_MPP_REFINE; it++) {", "for (int it = 0; it < 0; it++) {"),
    "sky_weight_uniform": ("double w = dot3(nh, ld3(dirs + 3 * j));", "double w = 1.0;"),
    "sky_back_directions_counted": ("if (!(w > 0.0)) continue;", ""),
    "sky_lit_share_flipped": ("num += w * (1.0 - f);", "num += w * f;"),
    "sky_reference_obstructed": ("double sky = counts && P->svf ? P->svf[m * cpm + c] : 1.0;   /* reference: whole sky */\n"
                                 "                    g[nc++]",
                                 "double sky = P->svf ? P->svf[m * cpm + c] : 1.0;\n                    g[nc++]"),
    "sphere_radius_full_diagonal": ("*radius = 0.5 * sqrt(dot3(dg, dg));\n}\n\nstatic v3 unit_normal",
                                    "*radius = sqrt(dot3(dg, dg));\n}\n\nstatic v3 unit_normal"),
    "depth_origin_shifted": ("V->znear = dot3(centre, V->d) - radius;", "V->znear = dot3(centre, V->d) - 0.25 * radius;"),
    "mpp_first_maximum_only": ("        if (!(p[q] >= p[q - 1]) || (q < OR_MPP_GRID && !(p[q] >= p[q + 1]))) continue;",
                               "        if (best > 0.0) break;\n"
                               "        if (!(p[q] >= p[q - 1]) || (q < OR_MPP_GRID && !(p[q] >= p[q + 1]))) continue;"),
}

PINS = [
    (zpins.test_zenith_depths_of_horizontal_planes, {}),
    (zpins.test_oblique_depths_of_planes_facing_the_sun, {}),
    (pins.test_c1_matches_exact_ray_casting, {}),
    (pins.test_c1_loss_closed_form, {"d_poa": 100.0, "want": 0.04670964}),
    (pins.test_string_power_is_best_operating_current, {}),
    (pins.test_fill_rule_covers_each_centre_once, {"seed": 0, "x0": 10.5, "y0": 7.5, "step": 4.0, "jitter": 0.0}),
    (pins.test_fill_rule_covers_each_centre_once, {"seed": 1, "x0": 10.5, "y0": 7.5, "step": 3.0, "jitter": 0.6}),
    (pins.test_depth_within_one_unit_of_exact_plane, {}),
    (pins.test_nearest_depth_wins_and_order_does_not_matter, {}),
    (pins.test_guard_band_clip_keeps_coverage_and_plane, {}),
    (pins.test_generator_alone_is_never_shaded, {}),
    (pins.test_back_lit_module_is_not_tested, {}),
    (pins.test_pole_shadow_length_on_flat_receiver, {"day": 355}),
    (pins.test_agrees_with_ray_casting_outside_band, {"seed": 21}),
    (tpins.test_pose_is_a_rigid_turn_about_the_pivot, {"kind": 2}),
    (tpins.test_pose_is_a_rigid_turn_about_the_pivot, {"kind": 1}),
    (tpins.test_two_axis_tracker_faces_the_sun, {}),
    (tpins.test_one_axis_tracker_faces_the_sun_as_its_axis_allows, {"axis": (0.6, -0.8, 0.0)}),
    (tpins.test_lone_tracker_is_never_shaded, {"kind": 2}),
    (tpins.test_tracker_shadow_agrees_with_ray_casting_outside_band, {"kind": 2}),
    (dpins.test_cell_voltage_matches_lambert_w, {"G": 700.0}),
    (dpins.test_uniform_string_is_cells_times_cell_maximum, {"G": 800.0}),
    (dpins.test_partial_shading_matches_brute_force, {"case": "one_shaded_substring"}),
    (dpins.test_partial_shading_matches_brute_force, {"case": "two_maxima_later_higher"}),
    (spins.test_wall_matches_the_infinite_wall_closed_form, {"tilt": 0.0, "north": True}),
    (spins.test_wall_matches_the_infinite_wall_closed_form, {"tilt": 30.0, "north": True}),
    (spins.test_sky_view_scales_only_the_diffuse, {}),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation site for {name} not found once"
    lib = O.build_variant(SRC.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    caught = []
    with O.use_library(lib):
        for fn, kw in PINS:
            try:
                fn(O, **kw)
            except (AssertionError, ValueError, IndexError):
                caught.append(fn.__name__)
                break
    assert caught, f"no pin fails when the oracle has mistake '{name}'"
