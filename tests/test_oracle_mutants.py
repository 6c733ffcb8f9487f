"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle source, plants one plausible mistake by a text
substitution, compiles the copy on the CPU and runs the pin and brute-force
suites against it in a subprocess.  The suites must fail for every mutant;
a mutant that passes would show a gap in the pins.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "raster_oracle.cpp")

MUTANTS = {
    "floor_not_trunc": ("*k = (int64_t)std::trunc(p);", "*k = (int64_t)std::floor(p);"),
    "round_not_trunc": ("*k = (int64_t)std::trunc(p);", "*k = (int64_t)std::llround(p);"),
    "fp32_product": ("double p = v * scale;", "double p = (double)((float)v * (float)scale);"),
    "four_neighbours": ("if (dx == 0 && dy == 0 && dz == 0) continue;", "if (dx == dy || dx == -dy) continue;"),
    "one_sided_neighbours": ("for (int64_t dx = -d; dx <= d; ++dx) {", "for (int64_t dx = -d; dx <= 0; ++dx) {"),
    "delta_ignored": ("const int64_t d = s->delta;", "const int64_t d = 1;"),
    "manhattan_as_chebyshev": ("if (s->metric == 1 && std::llabs(dx) + std::llabs(dy) + std::llabs(dz) > d) continue;",
                               ""),
    "manhattan_strict": ("std::llabs(dy) + std::llabs(dz) > d) continue;", "std::llabs(dy) + std::llabs(dz) >= d) continue;"),
    "z_neighbours_ignored": ("const int64_t dz_max = s->dims == 3 ? d : 0;", "const int64_t dz_max = 0;"),
    "z_not_projected": ("project_coord(point_coord(pts, dtype, s->dims, i, 2), s->scale, s->bound, &t.z)",
                        "project_coord(point_coord(pts, dtype, s->dims, i, 1), s->scale, s->bound, &t.z)"),
    "bound_3d_loose": ("kBound3d = 1048575.0;", "kBound3d = 2147483647.0;"),
    "square_one_corner_only": ("for (int64_t a = 0; a <= 1 && !by_square.count(t); ++a)",
                               "for (int64_t a = 0; a <= 0 && !by_square.count(t); ++a)"),
    "square_sum_strict": ("if (sum >= s->tau) {", "if (sum > s->tau) {"),
    "square_step_ignored": ("if (s->window) {", "if (false) {"),
    "chebyshev_square_too_small": ("for (int64_t dy = -d; dy <= d; ++dy) {", "for (int64_t dy = -d; dy < d; ++dy) {"),
    "tau_strict": ("if (it->second < s->tau && !by_square", "if (it->second <= s->tau && !by_square"),
    "mu_strict": ("if (cluster.size() >= s->mu)", "if (cluster.size() > s->mu)"),
    "label_is_max": ("if (t < lab) lab = t;", "if (lab < t) lab = t;"),
    "axes_swapped": ("project_coord(point_coord(pts, dtype, s->dims, i, 0), s->scale, s->bound, &t.x)",
                     "project_coord(point_coord(pts, dtype, s->dims, i, 0), s->scale, s->bound, &t.y)"),
    "duplicates_not_counted": ("else it->second += 1;", "else it->second = 1;"),
    "range_bound_loose": ("kBound2d = 2147483647.0;", "kBound2d = 2147483648.0;"),
    "f32_read_as_f64_lanes": ("return (double)((const float*)pts)[dims * i + c];",
                              "return (double)((const float*)pts)[i + c];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new)
    if name == "axes_swapped":  # also write y into x so the mutant stays consistent
        mutated = mutated.replace("project_coord(point_coord(pts, dtype, s->dims, i, 1), s->scale, s->bound, &t.y)",
                                  "project_coord(point_coord(pts, dtype, s->dims, i, 1), s->scale, s->bound, &t.x)")
    msrc = tmp_path / "mutant.cpp"
    msrc.write_text(mutated)
    sys.path.insert(0, ROOT)
    import oracle
    lib = oracle.compile_oracle(str(msrc), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, RASTER_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_brute.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
