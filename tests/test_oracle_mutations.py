"""The oracle's pins catch plausible mistakes.

Each case copies wipes_oracle.c to a temporary directory, plants one mistake
by replacing one expression, builds it, and runs the pins that are meant to
catch it against that build (WIPES_ORACLE_LIB).  The pins must fail.  The
mistakes live only in the temporary copy, on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wipes_oracle.c")

MUTATIONS = {
    "dropped_half_of_carrier": ("pe->kappa = 0.5 * (1.0 + cos(pe->phi));", "pe->kappa = (1.0 + cos(pe->phi));",
                                "test_pixel_sum_matches_poisson_closed_form"),
    "frequency_sign": ("pe->phi = s[SR_FX] * pe->dx + s[SR_FY] * pe->dy + s[SR_PH];",
                       "pe->phi = s[SR_FX] * pe->dx - s[SR_FY] * pe->dy + s[SR_PH];",
                       "test_pixel_sum_matches_poisson_closed_form or test_pixel_sum_gradient_closed_form"),
    "transposed_conic": ("s[SR_CA] = Syy / det;\n    s[SR_CB] = -Sxy / det;\n    s[SR_CC] = Sxx / det;",
                         "s[SR_CA] = Sxx / det;\n    s[SR_CB] = -Sxy / det;\n    s[SR_CC] = Syy / det;",
                         "test_pixel_sum_matches_poisson_closed_form or test_zero_frequency_is_gaussian_image"),
    "jacobian_column_sign": ("pj->J[2] = -cam->fx * uc / tz;", "pj->J[2] = cam->fx * uc / tz;",
                             "test_projection_off_axis_matches_linearised_pinhole"),
    "quaternion_order": ("R[1] = 2.0 * (x * y - w * z);", "R[1] = 2.0 * (x * y + w * z);",
                         "test_projection_off_axis_matches_linearised_pinhole"),
    "transmittance_update": ("T *= (1.0 - alpha);\n        dT += da", "T *= alpha;\n        dT += da",
                             "test_alpha_two_primitives_order_and_ties or test_alpha_termination_count"),
    "gradient_sign_of_mean": ("g[SG_MX] += dq * (-2.0 * Adx) + dphi * (-s[SR_FX]);",
                              "g[SG_MX] += dq * (2.0 * Adx) + dphi * (-s[SR_FX]);",
                              "test_fd_gradients_additive"),
    "scale_gradient_factor": ("dscale[3 * i + k] = 2.0 * pj.sc[k] * acc;", "dscale[3 * i + k] = pj.sc[k] * acc;",
                              "test_fd_gradients_alpha"),
    "binning_rounding": ("float x0 = ceilf((x - ex) - 0.5f), x1 = floorf((x + ex) - 0.5f);",
                         "float x0 = floorf((x - ex) - 0.5f), x1 = floorf((x + ex) - 0.5f);",
                         "test_binning_brute_force"),
    "binning_cross_term_sign": ("return fmaf(ca * dx, dx, fmaf(2.0f * cb * dx, dy, cc * dy * dy));",
                                "return fmaf(ca * dx, dx, fmaf(-2.0f * cb * dx, dy, cc * dy * dy));",
                                "test_binning_brute_force"),
    "binning_edge_slope": ("const float sy = -cb / cc, sx = -cb / ca;", "const float sy = -cb / ca, sx = -cb / cc;",
                           "test_binning_brute_force"),
    "covector_third_row_dropped": ("for (int k = 0; k < 3; ++k) dt[k] += (dJ3[k] - th[k] * dot) / tl;",
                                   "for (int k = 0; k < 3; ++k) dt[k] += 0.0 * (dJ3[k] - th[k] * dot) / tl;",
                                   "test_fd_gradients_covector"),
    "covector_inverse_transposed": (
        "for (int r = 0; r < 3; ++r) dfw[r] = Ai[3 * r] * g3[0] + Ai[3 * r + 1] * g3[1] + Ai[3 * r + 2] * g3[2];",
        "for (int r = 0; r < 3; ++r) dfw[r] = Ai[r] * g3[0] + Ai[3 + r] * g3[1] + Ai[6 + r] * g3[2];",
        "test_fd_gradients_covector or test_covector_frequency_gradient_closed_form"),
    "phase_sign": ("pe->phi = s[SR_FX] * pe->dx + s[SR_FY] * pe->dy + s[SR_PH];",
                   "pe->phi = s[SR_FX] * pe->dx + s[SR_FY] * pe->dy - s[SR_PH];",
                   "test_phase_pixel_sum_closed_form or test_phase_pointwise"),
    "phase_gradient_dropped": ("    g[SG_PH] += dphi;\n}", "    g[SG_PH] += 0.5 * dphi;\n}",
                               "test_phase_pixel_sum_closed_form or test_fd_gradients_phase"),
    "sh_basis_sign": ("v[1] = -c1 * y;", "v[1] = c1 * y;", "test_sh_basis_matches_scipy"),
    "sh_view_direction_gradient": ("for (int a = 0; a < 3; ++a) dm[a] += (du[a] - u[a] * dot) / dl;",
                                   "for (int a = 0; a < 3; ++a) dm[a] += du[a] / dl;",
                                   "test_fd_gradients_sh"),
    "support_counts_past_stop": ("T *= (1.0 - alpha);\n                if (T < P->T_min) break;",
                                 "T *= (1.0 - alpha);",
                                 "test_support_counts_brute_force"),
    "support_jump_bound_shrunk": ("jb[0] += fabs(s[SR_OP] * pe.w) *\n                                 fmax(",
                                  "jb[0] += 0.01 * fabs(s[SR_OP] * pe.w) *\n                                 fmax(",
                                  "test_tie_protocol"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new, selector = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must be unique: %s" % name
    mutated = tmp_path / "wipes_oracle.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-o",
                           str(lib), str(mutated), "-lm"])
    env = dict(os.environ, WIPES_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_oracle_variants.py"),
                        "-k", selector],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, "pins did not catch %s:\n%s" % (name, r.stdout[-2000:])
    assert "failed" in r.stdout
