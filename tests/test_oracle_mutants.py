"""The oracle's pins catch plausible mistakes.

Each case compiles a copy of ``oracle/bfs_oracle.c`` with one textual mistake
planted (a dropped term, a wrong index, LIFO instead of FIFO, an off-by-one
bound, a transposed operand) and checks that at least one pin fails. The
mistakes are planted in copies of the oracle on the CPU only.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_pins(so_path):
    """Run the pin sets on one oracle build in a child process (a crash counts as caught)."""
    return subprocess.run([sys.executable, "-m", "tests.run_pins", so_path], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)

MUTANTS = {
    "level_plus_two": ("levels[v] = levels[u] + 1;", "levels[v] = levels[u] + 2;"),
    "level_from_parent_missing": ("levels[v] = levels[u] + 1;", "levels[v] = 1;"),
    "parent_self": ("parents[v] = u;", "parents[v] = v;"),
    "parent_dropped": ("parents[v] = u;", ";"),
    "lifo_queue": ("int32_t u = queue[head++];", "int32_t u = queue[--tail]; head += 0;"),
    "last_neighbour_dropped": ("for (int64_t j = begin; j < end; ++j)", "for (int64_t j = begin; j + 1 < end; ++j)"),
    "first_neighbour_dropped": ("for (int64_t j = begin; j < end; ++j)", "for (int64_t j = begin + 1; j < end; ++j)"),
    "visited_test_inverted": ("if (levels[v] == -1) {", "if (levels[v] != 0) {"),
    "root_level_one": ("levels[root] = 0;", "levels[root] = 1;"),
    "root_parent_missing": ("parents[root] = (int32_t)root;", "parents[root] = -1;"),
    "row_end_wrong": ("end = offsets[u + 1];", "end = offsets[u] + 1;"),
    "operand_transposed": ("int32_t v = cols[j];", "int32_t v = (int32_t)(j % n);"),
    "init_zero": ("levels[v] = -1;\n        parents[v] = -1;", "levels[v] = 0;\n        parents[v] = -1;"),
    "min_parent_takes_max": ("if (u < parents[v]) parents[v] = (int32_t)u;",
                             "if (parents[v] == INT32_MAX || u > parents[v]) parents[v] = (int32_t)u;"),
    "min_parent_same_level": ("if (levels[v] != levels[u] + 1) continue;  /* the root",
                              "if (levels[v] != levels[u]) continue;  /* the root"),
    "min_parent_root_not_seeded": ("parents[root] = (int32_t)root;\n    for (int64_t u = 0; u < n; ++u) {\n        if (levels[u] < 0)",
                                   "for (int64_t u = 0; u < n; ++u) {\n        if (levels[u] < 0)"),
    "min_parent_last_arc_dropped": ("for (int64_t j = offsets[u]; j < offsets[u + 1]; ++j) {\n            const int32_t v = cols[j];\n            if (levels[v] != levels[u] + 1)",
                                    "for (int64_t j = offsets[u]; j + 1 < offsets[u + 1]; ++j) {\n            const int32_t v = cols[j];\n            if (levels[v] != levels[u] + 1)"),
    # The checkers (validate V1-V4, certify V2-V5).
    "check_level0_bound_dropped": ("if (levels[v] < 1 || u < 0", "if (u < 0"),
    "check_v3_dropped": ("if ((levels[v] == -1) != (parents[v] == -1)) {", "if (0) {"),
    "check_v2_root_parent_dropped": ("if (levels[root] != 0 || parents[root] != root) {", "if (levels[root] != 0) {"),
    "check_parent_level_dropped": ("levels[u] != levels[v] - 1 ||", ""),
    "check_arc_test_dropped": ("!has_arc(offsets, cols, u, (int32_t)v, rows_sorted)", "0"),
    "has_arc_search_off_by_one": ("return lo < offsets[u + 1] && cols[lo] == v;",
                                  "return lo + 1 < offsets[u + 1] && cols[lo] == v;"),
    "validate_v1_dropped": ("if (levels[v] != ref_levels[v]) {", "if (0) {"),
    "certify_v5_dropped": ("if (levels[v] == -1 || levels[v] > levels[u] + 1) {", "if (0) {"),
    "certify_v5_unreached_allowed": ("if (levels[v] == -1 || levels[v] > levels[u] + 1) {",
                                     "if (levels[v] > levels[u] + 1) {"),
    "certify_v5_skips_two": ("if (levels[v] == -1 || levels[v] > levels[u] + 1) {",
                             "if (levels[v] == -1 || levels[v] > levels[u] + 2) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    mutated = tmp_path / f"oracle_{name}.c"
    mutated.write_text(src.replace(old, new, 1))
    so = oracle.build(force=True, src=str(mutated), out=str(tmp_path / f"lib_{name}.so"))
    r = _run_pins(so)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout}"


def test_unmutated_copy_passes(tmp_path):
    src = open(oracle._SRC).read()
    p = tmp_path / "oracle_copy.c"
    p.write_text(src)
    r = _run_pins(oracle.build(force=True, src=str(p), out=str(tmp_path / "lib.so")))
    assert r.returncode == 0, r.stdout + r.stderr
