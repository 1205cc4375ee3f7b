"""The pins catch plausible mistakes: each mutant is the oracle with one
planted error (a flipped sign, a dropped term, a transposed operand, a wrong
tie rule ...), compiled on the CPU; at least one pin must fail against it."""
import ctypes as C
import os
import subprocess
import tempfile

import pytest

import test_oracle_pins as pins

MUTANTS = [
    ("Hessian xy sign", "out[3] = -h * xp * yp / D;", "out[3] = h * xp * yp / D;"),
    ("cut core dropped", "for (k = 0; k < 5; k++) d[k] = F * (Pa[k] - Ps[k]);",
     "for (k = 0; k < 5; k++) d[k] = F * Pa[k];"),
    ("rotation sign", "o[0] = c * v[0] - s * v[1];", "o[0] = c * v[0] + s * v[1];"),
    ("atan for atanh", "ay = pref * atanh(k * yp / (psi + q2 * S));",
     "ay = pref * atan(k * yp / (psi + q2 * S));"),
    ("q for q^2 in psi", "double psi = sqrt(q2 * (S * S + xp * xp) + yp * yp);",
     "double psi = sqrt(q * (S * S + xp * xp) + yp * yp);"),
    ("Hessian xx/yy transposed", "out[2] = h * (q2 * S * S + yp * yp + S * psi) / D;  /* xx */",
     "out[2] = h * (S * S + xp * xp + S * psi) / D;  /* xx */"),
    ("F missing", "F = s / (s - a);\n    }\n    double d[5]", "F = 1.0;\n    }\n    double d[5]"),
    ("distance ratio", "*out = 1.0 - comoving(zl, om, ol) / comoving(zs, om, ol);",
     "*out = comoving(zl, om, ol) / comoving(zs, om, ol);"),
    ("exact orientation term sign", "acc_product(L, by, ax, +1);", "acc_product(L, by, ax, -1);"),
    ("tie rule", "if (by != ay) return by < ay ? 1 : -1;", "if (by != ay) return by > ay ? 1 : -1;"),
    ("barycentric weight", "double ob = (ux[0] - ux[2]) * (py - uy[2]) - (uy[0] - uy[2]) * (px - ux[2]);",
     "double ob = (ux[0] - ux[2]) * (py - uy[2]) + (uy[0] - uy[2]) * (px - ux[2]);"),
    ("sigma not squared", "part += (ex * ex + ey * ey) / (C->sig[t] * C->sig[t]);",
     "part += (ex * ex + ey * ey) / C->sig[t];"),
    ("barycentre not a mean", "sx[i] = M > 0 ? mx / M : 0.0;", "sx[i] = M > 0 ? mx : 0.0;"),
    ("assignment tie", "if (bj < 0 || d2 < best) {", "if (bj < 0 || d2 <= best) {"),
    ("magnification sign", "double d = (1.0 - k) * (1.0 - k) - gg;",
     "double d = (1.0 - k) * (1.0 - k) + gg;"),
    ("convergence not halved", "double k = 0.5 * (hxx[i] + hyy[i]);", "double k = hxx[i] + hyy[i];"),
    ("shear component halved", "double g2 = hxy[i];", "double g2 = 0.5 * hxy[i];"),
    ("Newton update sign", "        cx = cx + sx;", "        cx = cx - sx;"),
    ("lens equation residual sign", "rx = bx - (cx - f * acc[0]);", "rx = bx - (cx + f * acc[0]);"),
    ("refinement skipped", "if (refine_max_iter > 0)", "if (refine_max_iter > 1000)"),
    ("potential log term without the core radius", "tl = w > 0.0 ? b0 * (1.0 - eps * eps) * w * 0.5 *",
     "tl = w > 0.0 ? b0 * (1.0 - eps * eps) * 0.5 *"),
    ("potential log term sign", "    return tx + ty - tl;", "    return tx + ty + tl;"),
    ("time delay geometric term", "out[at] = scale * (0.5 * (ex * ex + ey * ey) - dlsds * acc);",
     "out[at] = scale * ((ex * ex + ey * ey) - dlsds * acc);"),
    ("time-delay scale distances", "return cl * cs / ((cs - cl) * h0_si) * rad * rad / 86400.0;",
     "return cl * cs / (cs * h0_si) * rad * rad / 86400.0;"),
    ("Metropolis acceptance without the half", "d <= 0.0 || -2.0 * log(ul) > d",
     "d <= 0.0 || -log(ul) > d"),
    ("prior box ignored", "if (!(pr[i] >= lo[i] && pr[i] <= hi[i])) in = 0;", "(void)0;"),
    ("asymmetric proposal", "pr[i] = th[i] + step[i] * (2.0 * uw[i] - 1.0);",
     "pr[i] = th[i] + step[i] * (2.0 * uw[i] - 0.9);"),
    ("edge margin without the anti-diagonal", "if (i + 1 >= nx || j + 1 >= ny) continue;",
     "continue;"),
    ("edge margin without the segment clamp",
     "if (tt < 0) tt = 0;\n                if (tt > 1) tt = 1;\n                double qx = x1",
     "double qx = x1"),
    ("edge margin without the anti-diagonal's clamp",
     "if (tt < 0) tt = 0;\n                    if (tt > 1) tt = 1;\n                    double qx = xa",
     "double qx = xa"),
    ("edge margin skips the last row",
     "    for (j = 0; j < ny; j++) {\n        for (i = 0; i < nx; i++) {\n            /* edges from",
     "    for (j = 0; j < ny - 1; j++) {\n        for (i = 0; i < nx; i++) {\n            /* edges from"),
    ("edge margin deflection of the wrong vertex",
     "double y2 = grid_coord(gy0, j2, dy) - f * ay[id2];",
     "double y2 = grid_coord(gy0, j2, dy) - f * ay[id];"),
    ("edge margin without Dls/Ds on the anti-diagonal",
     "double xa = grid_coord(gx0, i + 1, dx) - f * ax[ia];",
     "double xa = grid_coord(gx0, i + 1, dx) - ax[ia];"),
    ("ellipticity conversion", "double or_eps_from_e(double e) { return e / (1.0 + sqrt(1.0 - e * e)); }",
     "double or_eps_from_e(double e) { return e / (1.0 + sqrt(1.0 + e * e)); }"),
]

PINS = [
    (pins.test_sis_deflection_is_einstein_radius, {}),
    (pins.test_circular_dpie_closed_form, {"a": 1.0, "s": 30.0}),
    (pins.test_elliptical_convergence_matches_surface_density, {}),
    (pins.test_hessian_is_derivative_of_deflection, {}),
    (pins.test_elliptical_deflection_by_independent_quadrature, {}),
    (pins.test_far_field_monopole, {}),
    (pins.test_rotation_covariance, {}),
    (pins.test_parameter_conversions, {}),
    (pins.test_distance_ratio_einstein_de_sitter, {}),
    (pins.test_orientation_sign_is_exact, {}),
    (pins.test_perturbed_orientation_tie_rule, {}),
    (pins.test_zero_lens_gives_one_image_at_the_source, {}),
    (pins.test_cored_isothermal_images_and_odd_multiplicity, {}),
    (pins.test_assignment_rules, {}),
    (pins.test_edge_margin_closed_forms, {}),
    (pins.test_source_chi2_zero_lens_closed_form, {}),
    (pins.test_image_chi2_zero_lens_closed_form, {}),
    (pins.test_derived_sis_closed_form, {}),
    (pins.test_derived_circular_dpie_shear_is_mean_minus_local_convergence, {"a": 0.5, "s": 30.0}),
    (pins.test_derived_det_is_jacobian_of_lens_mapping, {}),
    (pins.test_refine_sis_images_are_exact, {}),
    (pins.test_refine_cored_lens_matches_radial_roots, {}),
    (pins.test_refined_image_chi2_vanishes_for_noise_free_constraints, {}),
    (pins.test_potential_sis_is_b0_r, {}),
    (pins.test_potential_circular_dpie_closed_form, {"a": 0.5, "s": 30.0}),
    (pins.test_potential_gradient_is_deflection, {}),
    (pins.test_time_delay_sis_images, {}),
    (pins.test_time_delay_scale_einstein_de_sitter, {}),
    (pins.test_mcmc_zero_step_and_prior_rules, {}),
    (pins.test_mcmc_acceptance_threshold, {}),
    (pins.test_mcmc_samples_the_posterior, {}),
]


def build_mutant(src_text, path):
    from oracle import oracle as O
    with open(path + ".c", "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", *O.CFLAGS, path + ".c", "-o", path + ".so", "-lm"], check=True)
    return path + ".so"


@pytest.mark.parametrize("name,before,after", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(oracle, name, before, after):
    src = open(oracle.SRC).read()
    assert src.count(before) == 1, f"mutation site not found: {before}"
    with tempfile.TemporaryDirectory() as td:
        so = build_mutant(src.replace(before, after), os.path.join(td, "mut"))
        saved_lib, saved_path = oracle._lib, oracle.LIB
        oracle._lib, oracle.LIB = None, so
        failures = []
        try:
            oracle.lib()
            for fn, kw in PINS:
                try:
                    fn(oracle, **kw)
                except (AssertionError, ValueError, ZeroDivisionError, OverflowError) as e:
                    failures.append(fn.__name__)
        finally:
            oracle._lib, oracle.LIB = saved_lib, saved_path
    assert failures, f"no pin fails for the mutant '{name}'"
