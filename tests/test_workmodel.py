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


def test_molopt_basis_data_matches_table2():
    """the MOLOPT sets typed from Tables S2 and S3 have the composition (K and the
    l of each contracted function) that Table 2's counts are quoted for, and
    reproduce those counts"""
    from paper_1701_06588_amd import basis_molopt as bm
    g = json.load(open(GOLDEN))
    for name, key in (("H-DZVP", "H-DZVP"), ("O-DZVP", "O-DZVP")):
        b = bm.ORBITAL[name]
        assert len(b["exps"]) == g["basis"][key]["K"]
        assert b["l"] == g["basis"][key]["shells"]
        for deriv, dk in ((False, "Int"), (True, "Int+Dev")):
            os_c, shg_c = workmodel.contraction_counts(len(b["exps"]), b["l"], deriv)
            assert (os_c, shg_c) == (g["counts"][key]["OS"][dk], g["counts"][key]["SHG"][dk])


def test_molopt_sets_layout():
    """every function has one coefficient per exponent of its set, functions are
    grouped by l, and the spherical function counts are the sums of 2l+1"""
    import numpy as np
    from paper_1701_06588_amd import basis_molopt as bm
    st = bm.make_sets(np.zeros((4, 3)), list(bm.ORBITAL))
    assert list(st.nsgf()) == [5, 13, 29, 25]
    for s in range(st.n):
        ls = st.fun_l[st.fun_off[s]:st.fun_off[s] + st.nfun[s]]
        assert np.all(np.diff(ls) >= 0)
    for name, b in bm.ORBITAL.items():
        assert all(len(c) == len(b["exps"]) for c in b["coefs"])
        assert np.all(np.diff(b["exps"]) < 0)
    for name, rows in bm.AUX.items():
        e = [r[0] for r in rows]
        assert np.all(np.diff(e) < 0) and all(set(r[1]) <= {0, 1} for r in rows)
