"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of ``oracle/nrr_oracle.c`` (a text
substitution, compiled with gcc into a temporary directory, on the CPU) and
runs the pin suite against it in a subprocess; the suite must fail.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nrr_oracle.c")

MUTANTS = {
    "x_y_transposed": ("int64_t idx = (z * (int64_t)dims[1] + y) * (int64_t)dims[0] + x;",
                       "int64_t idx = (z * (int64_t)dims[1] + x) * (int64_t)dims[0] + y;"),
    "window_mean_dropped": ("double f = fbuf[i] - mean;", "double f = fbuf[i];"),
    "shift_sign_flipped": ("double v = ncc_at(tc, a, flt, dtype, dims, b, cx - h + dx, cy - h + dy,",
                           "double v = ncc_at(tc, a, flt, dtype, dims, b, cx - h - dx, cy - h - dy,"),
    "tie_takes_last": ("if (v > best) {", "if (v >= best) {"),
    "count_not_rounded": ("double k = floor(0.5 + (double)n_candidates * fraction);",
                          "double k = floor((double)n_candidates * fraction);"),
    "variance_ascending": ("if (a->key > b->key) return -1;\n    if (a->key < b->key) return 1;",
                           "if (a->key > b->key) return 1;\n    if (a->key < b->key) return -1;"),
    "flat_rule_one": ("if (!(ab > 0.0)) return 0.0;", "if (!(ab > 0.0)) return 1.0;"),
    "sqrt_dropped": ("return xx / sqrt(ab);", "return xx / ab;"),
    "range_too_tight": ("if (*hi > (n - 1 - h) - c) *hi = (n - 1 - h) - c;",
                        "if (*hi > (n - 2 - h) - c) *hi = (n - 2 - h) - c;"),
    "u16_key_unscaled": ("out_key[g] = (double)((int64_t)(b * b * b) * isq - isum * isum);",
                         "out_key[g] = (double)(isq - isum * isum);"),
    "block_half_size_off": ("int32_t h = (b - 1) / 2;\n    int64_t nb = (int64_t)b * b * b;\n#pragma omp parallel\n    {\n        double *tc = (double *)malloc(sizeof(double) * nb);\n        double *fb = (double *)malloc(sizeof(double) * nb);\n#pragma omp for schedule(dynamic, 1)\n        for (int64_t k = 0; k < n; ++k) {\n            int64_t cx",
                            "int32_t h = (b - 1) / 2 + 1;\n    int64_t nb = (int64_t)b * b * b;\n#pragma omp parallel\n    {\n        double *tc = (double *)malloc(sizeof(double) * nb);\n        double *fb = (double *)malloc(sizeof(double) * nb);\n#pragma omp for schedule(dynamic, 1)\n        for (int64_t k = 0; k < n; ++k) {\n            int64_t cx"),
}

# mistakes in the selection variants, caught by their own pin file
MUTANTS_EX = {
    "edges_counted_as_vertices": ("if (connectivity == 18 && steps > 2) continue;",
                                  "if (connectivity == 18 && steps > 3) continue;"),
    "mask_ignored": ("if (mask && !mask[(cz * dims[1] + cy) * (int64_t)dims[0] + cx]) continue;",
                     "if (0) continue;"),
    "count_over_all_candidates": ("const int64_t k = oracle_select_count(m, fraction);",
                                  "const int64_t k = oracle_select_count(n, fraction);"),
    "taken_not_marked": ("taken[g] = 1;\n        chosen[got++] = g;", "chosen[got++] = g;"),
    "faces_skip_z": ("for (int dz = -1; dz <= 1 && !blocked && connectivity; ++dz)",
                     "for (int dz = 0; dz <= 0 && !blocked && connectivity; ++dz)"),
}
# mistakes in the directional confidence
MUTANTS_CONF = {
    "border_difference_halved": ("    if (p[axis] == 0) {\n        hi[axis] = 1;\n        scale = 1.0;",
                                 "    if (p[axis] == 0) {\n        hi[axis] = 1;\n        scale = 0.5;"),
    "cross_term_sign": ("j[5] += gy * gz;", "j[5] -= gy * gz;"),
    "not_trace_normalised": ("out[6 * k + e] = tr > 0.0 ? conf[k] * j[e] / tr : 0.0;",
                             "out[6 * k + e] = tr > 0.0 ? conf[k] * j[e] : 0.0;"),
}
# mistakes in the per-axis (anisotropic) selection and search
MUTANTS_ANISO = {
    "aniso_window_axes_reversed": ("lo[a] = -w[a] > h[a] - c[a] ? -w[a] : h[a] - c[a];",
                                   "lo[a] = -w[2 - a] > h[a] - c[a] ? -w[2 - a] : h[a] - c[a];"),
    "aniso_centre_y_uses_x_half": (
        "out_centers[3 * i + 1] = (int32_t)(gy * stride[1] + (b[1] - 1) / 2);",
        "out_centers[3 * i + 1] = (int32_t)(gy * stride[1] + (b[0] - 1) / 2);"),
    "aniso_key_uses_cube": ("*key = (double)((int64_t)b[0] * b[1] * b[2] * isq - isum * isum);",
                            "*key = (double)((int64_t)b[0] * b[0] * b[0] * isq - isum * isum);"),
    "aniso_z_origin_uses_x_stride": ("gx * stride[0], gy * stride[1], gz * stride[2],",
                                     "gx * stride[0], gy * stride[1], gz * stride[0],"),
    "aniso_rows_along_y_too_short": (
        "for (int64_t y = 0; y < b[1]; ++y)\n            for (int64_t x = 0; x < b[0]; ++x) {\n                st +=",
        "for (int64_t y = 0; y < b[0]; ++y)\n            for (int64_t x = 0; x < b[0]; ++x) {\n                st +="),
    "aniso_at_displacement_sign": ("lo_f[a] = lo_r[a] + disp[3 * k + a];",
                                   "lo_f[a] = lo_r[a] - disp[3 * k + a];"),
    "aniso_at_x_half_everywhere": ("            const int64_t h = (b[a] - 1) / 2;\n            lo_r[a] = centers[3 * k + a] - h;",
                                   "            const int64_t h = (b[0] - 1) / 2;\n            lo_r[a] = centers[3 * k + a] - h;"),
    "aniso_tie_takes_last": (
        "if (v > best) {\n                        best = v;\n                        bd[0]",
        "if (v >= best) {\n                        best = v;\n                        bd[0]"),
}
# mistakes in the variants with per-axis sizes
MUTANTS_ANISO_EX = {
    "aniso_ex_edges_counted_as_vertices": ("connectivity == 18 ? 2 :", "connectivity == 18 ? 3 :"),
    "aniso_ex_mask_at_y_origin": ("cy = gy * stride[1] + (b[1] - 1) / 2,", "cy = gy * stride[1],"),
    "aniso_ex_z_neighbours_skipped": ("dz = j / 9 - 1;", "dz = (j / 9 - 1) * 0;"),
    "aniso_ex_mask_ignored": ("        if (mask && !mask[(cz * dims[1] + cy) * (int64_t)dims[0] + cx]) continue;\n        r[m++] = all[g];",
                              "        r[m++] = all[g];"),
}
PIN_FILES = {name: "test_oracle_pins.py" for name in MUTANTS}
PIN_FILES.update({name: "test_oracle_select_ex.py" for name in MUTANTS_ANISO_EX})
PIN_FILES.update({name: "test_oracle_aniso.py" for name in MUTANTS_ANISO})
PIN_FILES.update({name: "test_oracle_confidence.py" for name in MUTANTS_CONF})
PIN_FILES.update({name: "test_oracle_select_ex.py" for name in MUTANTS_EX})
MUTANTS.update(MUTANTS_EX)
MUTANTS.update(MUTANTS_CONF)
MUTANTS.update(MUTANTS_ANISO)
MUTANTS.update(MUTANTS_ANISO_EX)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "mutant.c"
    csrc.write_text(mutated)
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                           "-std=c11", str(csrc), "-o", str(lib), "-lm"])
    env = dict(os.environ, NRR_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", PIN_FILES[name])],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])
