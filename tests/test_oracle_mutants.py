"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies oracle/oracle.c, plants one plausible mistake (a flipped
tie-break, a dropped element, a wrong index or exponent, a half-open area
where the paper's is closed...), builds the copy in a temporary directory and
runs the full pin suite of tests/_pins.py against it.  The suite must fail.
"""
import os

import pytest

import oracle
from oracle import build as obuild
from tests import _pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "scan_rightmost_tie": ("if (A[t] < A[best])", "if (A[t] <= A[best])"),
    "scan_drops_last": ("for (int64_t t = l + 1; t <= r; t++)", "for (int64_t t = l + 1; t < r; t++)"),
    "combine_rightmost_tie": ("return p < q ? p : q;", "return p > q ? p : q;"),
    "st_exponent_short": ("int j = floor_log2(cnt);",
                          "int j = floor_log2(cnt) > 0 ? floor_log2(cnt) - 1 : 0;"),
    "st_drops_right_partial": ("if ((last_blk + 1) * b <= r)", "if (0)"),
    "block_st_no_doubling": ("cur[j] = j + half < nb ? (int32_t)better(A, prev[j], prev[j + half]) : prev[j];",
                             "cur[j] = prev[j];"),
    "block_st_wrong_offset": ("better(A, prev[j], prev[j + half]) : prev[j];",
                              "better(A, prev[j], prev[j + half - (half > 1)]) : prev[j];"),
    "contract_half_open": ("aq[s] = (int32_t)scan_argmin(A, pos[s], pos[s + 1]);",
                           "aq[s] = (int32_t)scan_argmin(A, pos[s], pos[s + 1] > pos[s] ? pos[s + 1] - 1 : pos[s]);"),
    "remap_right_off_by_one": ("Rc[t / 2] = (int32_t)(s - 1);",
                               "Rc[t / 2] = (int32_t)(s > 1 ? s - 2 : 0);"),
    "sort_tags_descending": ("return x->tag < y->tag ? -1 : 1;", "return x->tag < y->tag ? 1 : -1;"),
    "block_drops_last_element": ("pos[j] = (int32_t)scan_argmin(A, j * k, hi - 1);",
                                 "pos[j] = (int32_t)scan_argmin(A, j * k, hi - 2 >= j * k ? hi - 2 : j * k);"),
    "accepts_reversed_range": ("return 0 <= l && l <= r && r < n;", "return 0 <= l && r < n;"),
    "tour_children_descending": ("for (int64_t v = 0; v < N; v++)  /* increasing v: each list in id order */",
                                 "for (int64_t v = N - 1; v >= 0; v--)  /* decreasing */"),
    "tour_misses_up_steps": ("                if (top >= 0) {\n                    depth[len] = (int32_t)top;",
                             "                if (top >= 0 && top > 0) {\n                    depth[len] = (int32_t)top;"),
    "tour_first_is_last": ("                node[len] = (int32_t)stack_node[top];\n                    len++;",
                           "                node[len] = (int32_t)stack_node[top];\n                    first[stack_node[top]] = (int32_t)len;\n                    len++;"),
    "answer_skips_first": ("int64_t best = aq[Lc[i]];\n        for (int64_t s = (int64_t)Lc[i] + 1;",
                           "int64_t best = aq[Rc[i]];\n        for (int64_t s = (int64_t)Lc[i] + 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = obuild.build(str(mut), str(tmp_path / "liboracle_mut.so"))
    orc = oracle.Oracle(oracle.load(so))
    with pytest.raises((AssertionError, IndexError, ValueError)):
        _pins.run_all(orc)
