"""Plant plausible mistakes in copies of the oracle and check the pins catch them.

Each mutant is the oracle's C source with one textual change (a flipped sign,
a dropped or scaled carry, a wrong index or length, a transposed operand, an
imprecise constant, a wrong level order), compiled with gcc into a temporary
directory.  Every mutant must fail at least one pin of ``oracle_pins``; the
pins run in a child process so that a mutant which corrupts memory fails
loudly instead of taking the test runner down.  Everything here runs on the
CPU.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

RUNNER = r"""
import sys
sys.path[:0] = [{root!r}, {here!r}]
import oracle, oracle_pins
orc = oracle.Oracle({lib!r})
failed = []
for pin in oracle_pins.ALL_PINS:
    try:
        pin(orc)
    except Exception as e:
        failed.append(pin.__name__)
print("FAILED_PINS", ",".join(failed))
"""

MUTANTS = {
    "detail_sign": ("out[(na + m) * so] = s * (x1 - x0);", "out[(na + m) * so] = s * (x0 - x1);"),
    "carry_scaled": ("if (n & 1) out[pairs * so] = in[(n - 1) * si]; /* carry, unscaled    */",
                     "if (n & 1) out[pairs * so] = s * in[(n - 1) * si];"),
    "synthesis_phase_swap": ("out[(2 * m) * so] = s * (a - d);", "out[(2 * m) * so] = s * (a + d);"),
    "synthesis_carry_scaled": ("if (n & 1) out[(n - 1) * so] = in[pairs * si]; /* carry, unscaled    */",
                               "if (n & 1) out[(n - 1) * so] = s * in[pairs * si];"),
    "recursion_floor": ("fast_analysis_level(tmp, 1, y, 1, cur);\n        cur = (cur + 1) / 2;",
                        "fast_analysis_level(tmp, 1, y, 1, cur);\n        cur = cur / 2;"),
    "synthesis_operands_transposed": ("const double a = in[m * si];\n        const double d = in[(na + m) * si];",
                                      "const double d = in[m * si];\n        const double a = in[(na + m) * si];"),
    "2d_sizes_transposed": ("ch = (ch + 1) / 2;\n        cw = (cw + 1) / 2;",
                            "ch = (cw + 1) / 2;\n        cw = (ch + 1) / 2;"),
    "2d_width_floor": ("ch = (ch + 1) / 2;\n        cw = (cw + 1) / 2;",
                       "ch = (ch + 1) / 2;\n        cw = cw / 2;"),
    "2d_inverse_sizes": ("lh[j] = (lh[j - 1] + 1) / 2;", "lh[j] = lh[j - 1] / 2;"),
    "imprecise_constant": ("return sqrt(0.5);", "return 0.70710678;"),
    "inverse_level_order": ("for (int j = levels; j >= 1; --j) {\n        const int64_t cur = len[j - 1];\n        memcpy(tmp, x, (size_t)cur * sizeof(double));",
                            "for (int j = 1; j <= levels; ++j) {\n        const int64_t cur = len[j - 1];\n        memcpy(tmp, x, (size_t)cur * sizeof(double));"),
    "direct_tap_sign": ("b1[0] = s;  b1[1] = -s;", "b1[0] = -s; b1[1] = s;"),
    "direct_wrong_phase": ("out[m] = y0[2 * m + 1];", "out[m] = y0[2 * m];"),
    "shrink_threshold_level_order": ("c[i] = shrink_value(c[i], mode, thr[j - 1]);",
                                     "c[i] = shrink_value(c[i], mode, thr[levels - j]);"),
    "shrink_soft_sign": ("return d > 0.0 ? m : -m;", "return d > 0.0 ? -m : m;"),
    "shrink_2d_ll_included": ("if (r >= lh[j] || q >= lw[j])", "if (r >= 0)"),
    "shrink_2d_only_hh": ("if (r >= lh[j] || q >= lw[j])", "if (r >= lh[j] && q >= lw[j])"),
    "2d_row_skips_last": ("for (int64_t r = 0; r < ch; ++r) {            /* rows (width)   */",
                          "for (int64_t r = 0; r < ch - 1; ++r) {            /* rows (width)   */"),
    "l1_loss_ll_factor": ("l += 0.5 * *v * *v;", "l += *v * *v;"),
    "l1_ll_treated_as_detail": ("if (r < hL && q < wL) {", "if (r < hL && q < wL && 0) {"),
    "l1_detail_gradient_sign": ("*v = *v > 0.0 ? 1.0 : (*v < 0.0 ? -1.0 : 0.0);",
                                "*v = *v > 0.0 ? -1.0 : (*v < 0.0 ? 1.0 : 0.0);"),
    "3d_depth_floor": ("cd = (cd + 1) / 2;", "cd = cd / 2;"),
    "3d_z_pass_skipped": ("lines_3d(v, h, w, cd, ch, cw, 2, 0);", "/* z pass dropped */"),
    "3d_inverse_sizes": ("ld[j] = (ld[j - 1] + 1) / 2;", "ld[j] = ld[j - 1] / 2;"),
    "3d_inverse_y_skipped": ("lines_3d(v, h, w, ld[j - 1], lh[j - 1], lw[j - 1], 1, 1);", "/* y pass dropped */"),
    "3d_y_lines_plane_stride_as_row": ("else if (axis == 1) base = (q / cw) * h * w + (q % cw);",
                               "else if (axis == 1) base = (q / cw) * w + (q % cw);"),
    "3d_inverse_region_one_level_late": ("lines_3d(v, h, w, ld[j - 1], lh[j - 1], lw[j - 1], 2, 1);",
                                         "lines_3d(v, h, w, ld[j - 1], lh[j], lw[j - 1], 2, 1);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    src = open(oracle._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path_c = os.path.join(tmp_path, "mutant.c")
    with open(path_c, "w") as f:
        f.write(mutated)
    lib = oracle.build(force=True, src=path_c, out=os.path.join(tmp_path, "libmutant.so"))
    code = RUNNER.format(root=ROOT, here=HERE, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, OMP_NUM_THREADS="2"))
    if r.returncode != 0:
        return  # the mutant crashed or raised outside a pin: a loud failure
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED_PINS")][0]
    caught = [t for t in line.split(" ", 1)[1].split(",") if t] if " " in line else []
    assert caught, f"mutant {name} passed every pin"
