"""The pins catch plausible mistakes: each case plants one mistake in a copy of the oracle's
source (never in the oracle itself), builds it, and runs the pins that should notice, which
must then fail.  This checks the pins, not the oracle: a pin that a wrong oracle passes would
be no pin at all."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (what goes wrong, text in qed_oracle.c, its replacement, the pins that must fail)
MUTANTS = [
    ("emission density without its F2 term",
     "(F1 + 1.5 * delta * chi * zq * F2);", "(F1);",
     ["tests/test_oracle_rates.py"]),
    ("pair density with the brace's sign flipped",
     "(F1 - 1.5 * chi_g * zp * F2);", "(F1 + 1.5 * chi_g * zp * F2);",
     ["tests/test_oracle_rates.py"]),
    ("modified generator evaluating the density at r1 instead of r1^3",
     "  double delta = r1 * r1 * r1;\n  return 3.0 * r1 * r1 *",
     "  double delta = r1;\n  return 3.0 * r1 * r1 *",
     ["tests/test_oracle_generators.py::test_modified_generator_reproduces_spectrum"]),
    ("chi with (p.E)^2 added instead of subtracted",
     "double r = v0 * v0 + v1 * v1 + v2 * v2 - pe * pe;",
     "double r = v0 * v0 + v1 * v1 + v2 * v2 + pe * pe;",
     ["tests/test_oracle_kinematics.py"]),
    ("Boris rotation in the wrong sense",
     "t[i] = q * 0.5 * h * B[i] / g;", "t[i] = -q * 0.5 * h * B[i] / g;",
     ["tests/test_oracle_kinematics.py"]),
    ("Boris push missing its second half step in E",
     "for (int i = 0; i < 3; ++i) p[i] = pl[i] + q * 0.5 * h * E[i];",
     "for (int i = 0; i < 3; ++i) p[i] = pl[i];",
     ["tests/test_oracle_kinematics.py"]),
    ("Philox multiplier mistyped",
     "(uint64_t)0xD2511F53u * (uint64_t)c0", "(uint64_t)0xD2511F55u * (uint64_t)c0",
     ["tests/test_oracle_rng.py"]),
    ("Schwinger exponent exp(-pi E) instead of exp(-pi E_S / E)",
     "exp(-OR_PI / e)", "exp(-OR_PI * e)",
     ["tests/test_oracle_schwinger.py"]),
    ("children left one sub-step too much of the step",
     "c.tau = (double)(left) * h;", "c.tau = (double)(left + 1) * h;",
     ["tests/test_oracle_same_step.py::test_photon_children_move_through_the_rest_of_the_step"]),
    ("thinning factor inverted",
     "w_live / w_kept", "w_kept / w_live",
     ["tests/test_oracle_thinning.py::test_weight_conserved_and_survivors_untouched"]),
    ("lepton time-step bound with 140 for 14",
     "kappa * 14.0 * (2.0 * OR_PI * eps_r)", "kappa * 140.0 * (2.0 * OR_PI * eps_r)",
     ["tests/test_oracle_kinematics.py"]),
    ("Ex sampled on the nodes instead of the half-nodes",
     "{{0.5, 0, 0},   {0, 0.5, 0}", "{{0.0, 0, 0},   {0, 0.5, 0}",
     ["tests/test_oracle_kinematics.py"]),
    ("emission without recoil",
     "for (int d = 0; d < 3; ++d) mom[d] = mom[d] - c.p[d];",
     "for (int d = 0; d < 3; ++d) mom[d] = mom[d];",
     ["tests/test_oracle_step.py"]),
    ("Schwinger rate with the Compton length cubed instead of to the fourth",
     "pow(eps_r, 4.0)", "pow(eps_r, 3.0)",
     ["tests/test_oracle_schwinger.py"]),
    ("photon chi without the photon energy factor",
     "return kabs * H * eps_r;", "return H * eps_r;",
     ["tests/test_oracle_kinematics.py", "tests/test_oracle_rates.py"]),
    ("pair probability scaled by |k| instead of divided",
     "(chi_g / kabs) * (delta_e - 1.0)", "(chi_g * kabs) * (delta_e - 1.0)",
     ["tests/test_oracle_rates.py"]),
    ("pair leptons not inheriting the photon's magnetic field for the rest of the step",
     "e.B[d] = pos.B[d] = B[d];", "e.B[d] = pos.B[d] = 0.0;",
     ["tests/test_oracle_same_step.py::test_pair_leptons_turn_through_the_rest_of_the_step"]),
    ("standard generator's W without the ln 2 of d delta / du",
     "return or_rate_emission(a->t, a->backend, d, a->chi, a->gamma, a->dtfac) * log(2.0) * d /",
     "return or_rate_emission(a->t, a->backend, d, a->chi, a->gamma, a->dtfac) * d /",
     ["tests/test_oracle_generator_comparison.py"]),
    ("lepton position advanced by p instead of p / gamma",
     "x[d] += h * mom[d] / gamma;", "x[d] += h * mom[d];",
     ["tests/test_oracle_step.py::test_leptons_gyrate_on_their_larmor_circle"]),
    ("Schwinger pair placed on the cell's diagonal (one uniform for two axes)",
     "((double)o[0] + 0.5) * 0x1p-32, ((double)o[1] + 0.5) * 0x1p-32,",
     "((double)o[0] + 0.5) * 0x1p-32, ((double)o[0] + 0.5) * 0x1p-32,",
     ["tests/test_oracle_schwinger.py"]),
    ("photon chi with the sign of k x B flipped in one component",
     "double v0 = E[0] + (n1 * B[2] - n2 * B[1]);", "double v0 = E[0] - (n1 * B[2] - n2 * B[1]);",
     ["tests/test_oracle_kinematics.py"]),
    ("rotating field turning the other way",
     "      E[1] = f->amp * sin(ph);", "      E[1] = -f->amp * sin(ph);",
     ["tests/test_oracle_kinematics.py"]),
    ("emitted photon along the lepton's x axis only",
     "c.p[d] = (eps / pabs) * mom[d];", "c.p[d] = (eps / pabs) * mom[0];",
     ["tests/test_oracle_step.py"]),
    ("Schwinger cell field not averaged over its four samples",
     "const double ex = 0.25 * (or_grid_at(f->grid[0]",
     "const double ex = 0.5 * (or_grid_at(f->grid[0]",
     ["tests/test_oracle_schwinger.py"]),
    ("generator factor not raising the children's weight",
     "return fg > 1.0 ? fg : 1.0;", "return 1.0;",
     ["tests/test_oracle_generator_factor.py"]),
    ("a sub-step kept although its end state breaks Eq. (29)",
     "      if (h > dtq) {\n", "      if (0 && h > dtq) {\n",
     ["tests/test_oracle_stats.py::test_slowed_leptons_refine_their_substeps"]),
    ("refined sub-steps that do not add up to the step",
     "          left *= 2;", "          left *= 3;",
     ["tests/test_oracle_stats.py::test_slowed_leptons_refine_their_substeps"]),
    ("photon-energy histogram in natural logarithms",
     "floor(10.0 * (log10(eps) + 8.0))", "floor(10.0 * (log(eps) + 8.0))",
     ["tests/test_oracle_stats.py::test_photon_histogram_and_energy_match_the_emitted_photons"]),
    ("largest pair probability taken over every decision",
     "if (r2 < P && P > s->max_p_pair)", "if (P > s->max_p_pair)",
     ["tests/test_oracle_stats.py::test_largest_pair_probability_is_that_of_a_pair_made"]),
    ("cell thinning that scales survivors by the group's count ratio, not its weight ratio",
     "      const double f = W / K;", "      const double f = (double)m / (double)kept;",
     ["tests/test_oracle_thin_cells.py"]),
    ("cell thinning that groups by x alone",
     "  return (b[2] * nb[1] + b[1]) * nb[0] + b[0];", "  return b[0];",
     ["tests/test_oracle_thin_cells.py"]),
    ("cell thinning that lets an empty group lose its weight",
     "      if (kept == 0) { /* the group keeps its weight in its smallest draw */",
     "      if (kept < 0) { /* the group keeps its weight in its smallest draw */",
     ["tests/test_oracle_thin_cells.py"]),
    ("reverse-mode recoil by the sum of the runs' photons, not their mean",
     "mom[d] = mom[d] - rec[d] / (double)R;", "mom[d] = mom[d] - rec[d];",
     ["tests/test_oracle_generator_forms.py::test_reverse_emission_conserves_the_weighted_momentum"]),
    ("reverse-mode runs that share one draw",
     "((uint32_t)substep & 0xFFFFu) | ((uint32_t)run << 24),", "((uint32_t)substep & 0xFFFFu),",
     ["tests/test_oracle_generator_forms.py::test_reverse_emission_runs_are_independent_and_unbiased"]),
    ("reverse-mode photon that keeps its whole weight after a partial decay",
     "if (m > 0) wcur = wc * (double)(R - m);", "if (m > 0) wcur = wcur;",
     ["tests/test_oracle_generator_forms.py::test_reverse_pairs_conserve_the_photon_weight"]),
    ("deterministic factor without a phase (the first event always makes a child)",
     "return ((uint64_t)e + phi) % (uint64_t)F == 0;", "return (uint64_t)e % (uint64_t)F == 0;",
     ["tests/test_oracle_generator_forms.py::test_deterministic_factor_is_unbiased"]),
    ("deterministic factor whose phase changes along the parent's life",
     "uint32_t ctr[4] = {0u, 12u << 16,", "uint32_t ctr[4] = {e / 3u, 12u << 16,",
     ["tests/test_oracle_generator_forms.py::test_deterministic_every_fourth_event_with_one_phase"]),
    ("cell thinning with the global thinning's draw purpose",
     "uint32_t ctr[4] = {(uint32_t)step, 11u << 16,", "uint32_t ctr[4] = {(uint32_t)step, 4u << 16,",
     ["tests/test_oracle_thin_cells.py"]),
]


@pytest.mark.parametrize("what,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_a_planted_mistake(tmp_path, what, old, new, pins):
    src = open(os.path.join(ORACLE, "qed_oracle.c")).read()
    assert src.count(old) == 1, "the mutation site must be unique"
    (tmp_path / "qed_oracle.c").write_text(src.replace(old, new))
    shutil.copy(os.path.join(ORACLE, "qed_oracle.h"), tmp_path / "qed_oracle.h")
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", "-o", str(lib),
                    str(tmp_path / "qed_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, QED_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *pins], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode != 0, f"no pin noticed: {what}\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "error" in r.stdout.lower(), r.stdout[-2000:]
