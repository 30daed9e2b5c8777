"""The work model reproduces the contraction counts of Table 2 (golden fixture)."""
import json
import os

from paper_1701_06588_amd import workmodel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_counts.json")


def test_table2_counts():
    g = json.load(open(GOLDEN))
    for name, spec in g["basis"].items():
        for deriv, key in ((False, "Int"), (True, "Int+Dev")):
            os_c, shg_c = workmodel.contraction_counts(spec["K"], spec["shells"], deriv)
            assert os_c == g["counts"][name]["OS"][key], (name, key)
            assert shg_c == g["counts"][name]["SHG"][key], (name, key)


def test_pair_bytes():
    assert workmodel.pair_bytes(0, 0, False) == 8 + 16
    assert workmodel.pair_bytes(4, 4, True) == 8 * 81 * 4 + 16
