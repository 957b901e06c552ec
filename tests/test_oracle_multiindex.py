"""Pins the multi-index sets: the worked D=2, p=2 example of section 2, the
C(D+p-1, D) counts, the PLIMIT table of section 6, and brute-force enumeration."""
import itertools
import json
import math
import os

import pytest

from oracle.multiindex import multi_indices, num_terms, plimit_for

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_d2_p2():
    g = json.load(open(os.path.join(GOLD, "worked_example_d2p2.json")))
    got = multi_indices(g["D"], g["p"])
    assert [list(a) for a in got] == g["o_Dp_terms"]
    assert len(got) == g["o_Dp_count"]
    # the O(p^D) tensor set keeps every alpha with alpha_d < p
    pd = set(itertools.product(range(g["p"]), repeat=g["D"]))
    assert pd == {tuple(a) for a in g["o_pD_terms"]}
    assert len(pd) == g["o_pD_count"] == g["p"] ** g["D"]


def test_plimit_table_and_counts():
    g = json.load(open(os.path.join(GOLD, "plimit.json")))
    for D, P in g["plimit"].items():
        assert plimit_for(int(D)) == P
    for D, C in g["terms_at_plimit"].items():
        assert num_terms(int(D), plimit_for(int(D))) == C
        assert len(multi_indices(int(D), plimit_for(int(D)))) == C


@pytest.mark.parametrize("D,p", [(1, 6), (2, 8), (3, 6), (4, 5), (5, 4), (8, 3)])
def test_brute_force_enumeration(D, p):
    mis = multi_indices(D, p)
    brute = {a for a in itertools.product(range(p), repeat=D) if sum(a) < p}
    assert set(mis) == brute
    assert len(mis) == len(brute) == math.comb(D + p - 1, D)
    degs = [sum(a) for a in mis]
    assert degs == sorted(degs)                       # graded
    for deg in range(p):                              # decreasing lex inside a degree
        block = [a for a in mis if sum(a) == deg]
        assert block == sorted(block, reverse=True)
    for q in range(1, p):                             # prefix property
        assert mis[: num_terms(D, q)] == multi_indices(D, q)
