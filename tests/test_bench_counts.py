"""The per-row work counts bench.py prices its roofline fractions on (the
window contraction done dimension by dimension; the factored contraction
shared by the fast input's values), checked against values written out by
hand and against counts of the multiply-adds a literal loop nest issues."""
import itertools
import math
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))
import bench  # noqa: E402


def _fma_count_nested(L):
    # a loop nest that contracts the innermost dimension first: one
    # multiply-add per cell of every partial window it forms
    n = 0
    for k in range(len(L), 0, -1):
        n += math.prod(L[:k])
    return n


@pytest.mark.parametrize("L", [(3, 3, 3, 3, 3), (5, 5, 2), (6, 6, 3), (2, 2, 3, 3, 3, 3, 3), (13, 13), (7,)])
def test_contraction_count_is_the_nested_loop_count(L):
    plan = {"window": list(L) + [0] * (8 - len(L)), "W": math.prod(L)}
    assert bench.contraction_flops_per_row(plan) == 2 * _fma_count_nested(L)


def test_contraction_count_room_and_unicycle():
    # 3^5: 2 (243 + 81 + 27 + 9 + 3); 5 x 5 x 2: 2 (50 + 25 + 5)
    assert bench.contraction_flops_per_row({"window": [3] * 5, "W": 243}) == 726
    assert bench.contraction_flops_per_row({"window": [5, 5, 2], "W": 50}) == 160


@pytest.mark.parametrize("L,nf", [((5, 5, 2), 9), ((6, 6, 3), 9), ((5, 5, 2), 1), ((4, 3, 2), 5), ((2, 3, 4, 2), 3)])
def test_factored_count_by_enumeration(L, nf):
    # walk the factored sweep's loop nest for one state and one slow
    # combination, counting multiply-adds: every outer level D (0 .. n-2)
    # accumulates U partial sums once per index tuple (k_0 .. k_D); then
    # each of the nf fast inputs sums L_last of the U partial sums
    U = L[-1] + 3
    fma = 0
    outer = L[:-1]
    for D in range(len(outer)):
        for _ in itertools.product(*[range(x) for x in outer[:D + 1]]):
            fma += U
    per_row = 2 * fma / nf + 2 * L[-1]
    plan = {"window": list(L), "W": math.prod(L)}
    assert bench.factored_flops_per_row(plan, nf) == pytest.approx(per_row)


def test_factored_count_unicycle_values():
    # 2 * 5 * 5 * (5 + 1) / 9 + 2 * 2 and 2 * 6 * 6 * (6 + 1) / 9 + 2 * 3
    assert bench.factored_flops_per_row({"window": [5, 5, 2], "W": 50}, 9) == pytest.approx(300 / 9 + 4)
    assert bench.factored_flops_per_row({"window": [6, 6, 3], "W": 108}, 9) == pytest.approx(504 / 9 + 6)
