"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of oracle/oracle.c (a dropped
factor, a wrong sign, a transposed index, a non-strict cutoff, a lost
neighbour layer, ...), compiles the copy into a temporary library, and runs
the pin tests (tests/test_oracle_pins.py) against it in a child process.
Every planted mistake must make at least one pin fail.  The altered copies
live only in pytest's temporary directory; the oracle itself is untouched.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement, which occurrence (0-based), how many
# occurrences the text has).  The kernel formulas appear twice: first in
# oracle_kernel (from r), then in the sweep's kernel (from r^2).
MUTANTS = [
    ("kernel_inner_sign_from_r", "6.0 * q * q * q - 6.0 * q * q + 1.0", "6.0 * q * q * q + 6.0 * q * q + 1.0", 0, 2),
    ("kernel_inner_sign_from_d2", "6.0 * q * q * q - 6.0 * q * q + 1.0", "6.0 * q * q * q + 6.0 * q * q + 1.0", 1, 2),
    ("kernel_outer_factor_two", "*W = 2.0 * sigma * omq * omq * omq;", "*W = sigma * omq * omq * omq;", 1, 2),
    ("kernel_outer_derivative_sign", "*dWdr = -(6.0 * sigma / h) * omq * omq;", "*dWdr = (6.0 * sigma / h) * omq * omq;", 1, 2),
    ("kernel_inner_derivative_swapped", "(18.0 * q * q - 12.0 * q)", "(12.0 * q * q - 18.0 * q)", 1, 2),
    ("kernel_norm_h_squared_from_r", "8.0 / (M_PI * h * h * h)", "8.0 / (M_PI * h * h)", 0, 2),
    ("kernel_norm_h_squared_from_d2", "8.0 / (M_PI * h * h * h)", "8.0 / (M_PI * h * h)", 1, 2),
    ("one_minus_q_missing_factor", "(h * h - d2) / (h * (h + r))", "(h * h - d2) / (h * h)", 0, 1),
    ("sweep_cutoff_not_strict", "if (!(d2 < rc2)) continue;", "if (!(d2 <= rc2)) continue;", 0, 2),
    ("brute_cutoff_not_strict", "if (!(d2 < rc2)) continue;", "if (!(d2 <= rc2)) continue;", 1, 2),
    ("sweep_lost_lower_z_layer", "for (int dz = -1; dz <= 1; ++dz) {", "for (int dz = 0; dz <= 1; ++dz) {", 0, 2),
    ("sweep_self_not_excluded", "if (j == i) continue;\n                        r_cand += 1;",
     "r_cand += 1;", 0, 1),
    ("sweep_gradient_sign", "const double ddx = xi - (double)x[j];", "const double ddx = (double)x[j] - xi;", 0, 2),
    ("cell_index_transposed", "cell[i] = ix + dims[0] * (iy + dims[1] * iz);",
     "cell[i] = iy + dims[1] * (ix + dims[0] * iz);", 0, 1),
    ("scatter_order_descending", "for (int64_t i = 0; i < n; ++i) {\n        const int32_t c = cell[i];",
     "for (int64_t i = n - 1; i >= 0; --i) {\n        const int32_t c = cell[i];", 0, 1),
    ("relative_coordinate_ignores_origin", "fmaf(-(float)ix, cell_w, x[i] - origin[0])",
     "fmaf(-(float)ix, cell_w, x[i])", 0, 1),
    ("sweep_ascale_signed", "r_a += wj * fabs(dW);", "r_a += wj * dW;", 0, 2),
    ("brute_ascale_signed", "r_a += wj * fabs(dW);", "r_a += wj * dW;", 1, 2),
    ("sweep_target_weight", "const double wj = (double)w[j];", "const double wj = (double)w[i];", 0, 2),
    ("sweep_gradient_not_over_r", "const double f = wj * dW / r;", "const double f = wj * dW;", 0, 2),
    ("sweep_cell_decode_axes_swapped", "iy = (c / nx) % ny", "iy = (c / ny) % nx", 0, 2),
    ("max_per_cell_ignored", "if (counts[c] > mc) mc = counts[c];", "if (counts[c] > mc) mc = 1;", 0, 1),
    # the timing-experiment kernels (Lennard-Jones, low- and high-FLOP)
    ("lj_attractive_sign", "double k = 4.0 * p->e0 * (u3 * u3 - u3);", "double k = 4.0 * p->e0 * (u3 * u3 + u3);",
     0, 1),
    ("lj_missing_four", "double k = 4.0 * p->e0 *", "double k = p->e0 *", 0, 1),
    ("lj_no_softening", " + p->eps * p->eps;", ";", 0, 1),
    ("lj_cube_as_square", "const double u3 = u * u * u;", "const double u3 = u * u;", 0, 1),
    ("lowflop_sign", "*K = dx + dy + dz;", "*K = dx + dy - dz;", 0, 1),
    ("lowflop_ascale_signed", "*A = fabs(dx) + fabs(dy) + fabs(dz);", "*A = dx + dy + dz;", 0, 1),
    ("highflop_changes_value", "k = fma(k, p->a, p->b);", "k = fma(k, p->a, p->a);", 0, 1),
    ("pairfn_sweep_self_included", "if (j == i) continue;\n                        double K, A;", "double K, A;",
     0, 1),
    ("pairfn_sweep_lost_upper_x_cell", "for (int dx = -1; dx <= 1; ++dx) {\n                    const int32_t cx = ix + dx;\n"
     "                    if (cx < 0 || cx >= nx) continue;\n                    const int64_t nc = cx + (int64_t)nx * (cy + (int64_t)ny * cz);\n"
     "                    for (int64_t k = offsets[nc]; k < offsets[nc + 1]; ++k) {\n                        const int64_t j = perm[k];\n"
     "                        if (j == i) continue;\n                        double K, A;",
     "for (int dx = -1; dx <= 0; ++dx) {\n                    const int32_t cx = ix + dx;\n"
     "                    if (cx < 0 || cx >= nx) continue;\n                    const int64_t nc = cx + (int64_t)nx * (cy + (int64_t)ny * cz);\n"
     "                    for (int64_t k = offsets[nc]; k < offsets[nc + 1]; ++k) {\n                        const int64_t j = perm[k];\n"
     "                        if (j == i) continue;\n                        double K, A;", 0, 1),
    ("pairfn_brute_reach_two_cells", "abs(jx - ix) > 1", "abs(jx - ix) > 2", 0, 1),
]


def _mutate(text, old, new, which, total):
    assert text.count(old) == total, f"oracle.c changed: {old!r} occurs {text.count(old)} times"
    at = -1
    for _ in range(which + 1):
        at = text.index(old, at + 1)
    return text[:at] + new + text[at + len(old):]


def _run_pins(lib):
    env = dict(os.environ, ORACLE_LIBRARY=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unaltered_copy_passes_the_pins(tmp_path):
    """Control: a copy built the same way, with nothing planted, passes."""
    lib = str(tmp_path / "liboracle_copy.so")
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-o", lib, SRC, "-lm"], check=True)
    rc, out = _run_pins(lib)
    assert rc == 0, out


def test_every_planted_mistake_fails_a_pin(tmp_path):
    text = open(SRC).read()
    libs = {}
    for name, old, new, which, total in MUTANTS:
        src = tmp_path / f"{name}.c"
        src.write_text(_mutate(text, old, new, which, total))
        lib = str(tmp_path / f"lib{name}.so")
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-fno-fast-math", "-o", lib, str(src), "-lm"], check=True)
        libs[name] = lib
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = dict(zip(libs, ex.map(_run_pins, libs.values())))
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mistakes no pin caught: {survivors}"
