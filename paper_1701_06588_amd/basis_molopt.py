"""MOLOPT orbital and LRI-MOLOPT auxiliary basis sets of the paper's
supplement (Tables S2-S8), as family sets: one set per element, every
contracted function of the set on the same exponents (Sec. III).

Orbital sets (Tables S2-S5): exponents and, per contracted function, its l and
its contraction coefficients (columns of the table, in the table's order, which
groups the functions by l). Auxiliary sets (Tables S6-S8) are uncontracted: per
exponent, the l values that carry one function each.

This module holds data only (no integral arithmetic), so both the GPU path and
the CPU oracle take their basis from here.
"""
from __future__ import annotations

import numpy as np

from . import inputs

# Table S2: H-DZVP-MOLOPT-GTH
H_DZVP = {
    "exps": [11.478000339908, 3.700758562763, 1.446884268432, 0.716814589696, 0.247918564176,
             0.066918004004, 0.021708243634],
    "l": [0, 0, 1],
    "coefs": [
        [0.024916243200, 0.079825490000, 0.128862675300, 0.379448894600, 0.324552432600, 0.037148121400,
         -0.001125195500],
        [-0.012512421400, -0.056449071100, 0.011242684700, -0.418587548300, 0.590363216700, 0.438703133000,
         -0.059693171300],
        [0.024510918200, 0.058140794100, 0.444709498500, 0.646207973100, 0.803385018200, 0.892971208700,
         0.120101316500],
    ],
}

# Table S3: O-DZVP-MOLOPT-GTH
O_DZVP = {
    "exps": [12.015954705512, 5.108150287385, 2.048398039874, 0.832381575582, 0.352316246455,
             0.142977330880, 0.046760918300],
    "l": [0, 0, 1, 1, 2],
    "coefs": [
        [-0.060190841200, -0.129597923300, 0.118175889400, 0.462964485000, 0.450353782600, 0.092715833600,
         -0.000255945800],
        [0.065738617900, 0.110885902200, -0.053732406400, -0.572670666200, 0.186760006700, 0.387201458600,
         0.003825849600],
        [0.036543638800, 0.120927648700, 0.251093670300, 0.352639910300, 0.294708645200, 0.173039869300,
         0.009726110600],
        [-0.034210557400, -0.120619770900, -0.213719464600, -0.473674858400, 0.484848376400, 0.717465919700,
         0.032498979400],
        [0.014807054400, 0.068186159300, 0.290576499200, 1.063344189500, 0.307656114200, 0.318346834400,
         -0.005771736600],
    ],
}

# Table S4: O-TZV2PX-MOLOPT-GTH
O_TZV2PX = {
    "exps": list(O_DZVP["exps"]),
    "l": [0, 0, 0, 1, 1, 1, 2, 2, 3],
    "coefs": [
        O_DZVP["coefs"][0],
        O_DZVP["coefs"][1],
        [0.041006765400, 0.080644802300, -0.067639801700, -0.435078312800, 0.722792798300, -0.521378340700,
         0.175643142900],
        O_DZVP["coefs"][2],
        O_DZVP["coefs"][3],
        [-0.000592640200, 0.009852349400, 0.001286509800, -0.021872639500, 0.530504764700, -0.436184043700,
         0.073329259500],
        O_DZVP["coefs"][4],
        [-0.013843410500, 0.016850210400, -0.186696332600, 0.068001578700, 0.911407510000, -0.333128530600,
         -0.405788515900],
        [0.002657486200, -0.007708463700, 0.378459897700, 0.819571172100, -0.075845376400, 0.386329438600,
         0.035062554400],
    ],
}

# Table S5: Cu-DZVP-MOLOPT-SR-GTH
CU_DZVP = {
    "exps": [5.804051150731, 2.947777593081, 1.271621207972, 0.517173767860, 0.198006620331, 0.061684232135],
    "l": [0, 0, 1, 1, 2, 2, 3],
    "coefs": [
        [0.020918100390, -0.106208582202, 0.307397740339, 0.240805274553, -0.798718095004, -0.738671023869],
        [0.045720931893, -0.094026024883, -0.110623536813, -0.742218346329, 2.208107372713, -1.720016262377],
        [-0.004381592772, 0.017185613995, -0.089805629814, 0.054415126660, 0.446326740476, 0.468516012555],
        [-0.021109803873, 0.020960301873, 0.233442747472, 0.369266430953, -1.405067129701, 1.042169799071],
        [0.275442696345, 0.351705110927, 0.331635969640, 0.259386540456, 0.151105835782, 0.030634833418],
        [-0.101811263028, -0.207670618594, -0.224161904198, 0.176105738988, 0.210534119173, 0.902456275117],
        [-0.016523760157, 0.055142365254, -0.286656089760, -0.502349311598, -0.508940020577, 0.682110135764],
    ],
}

# Tables S6-S8: LRI-MOLOPT auxiliary sets; per exponent the number of functions
# of each l (columns s, p, d, f, g, h, i), all 0 or 1
H_LRI = [
    (22.956000679816, [1, 0, 0, 0]), (11.437045132575, [1, 1, 0, 0]), (5.6981180297480, [1, 1, 1, 0]),
    (2.8388931498100, [1, 1, 1, 0]), (1.4143817790300, [1, 1, 1, 1]), (0.7046675275490, [1, 1, 1, 1]),
    (0.3510765846560, [1, 1, 1, 1]), (0.1749119456700, [1, 1, 1, 1]), (0.0871439169550, [1, 1, 1, 1]),
    (0.0434164872680, [1, 1, 1, 1]),
]
O_LRI = [
    (24.031909411024, [1, 0, 0, 0, 0]), (16.167926705922, [1, 0, 0, 0, 0]), (10.877281929506, [1, 1, 0, 0, 0]),
    (7.3178994639200, [1, 1, 1, 0, 0]), (4.9232568311730, [1, 1, 1, 1, 0]), (3.3122151985280, [1, 1, 1, 1, 0]),
    (2.2283561263540, [1, 1, 1, 1, 1]), (1.4991692049680, [1, 1, 1, 1, 1]), (1.0085947567100, [1, 1, 1, 1, 1]),
    (0.6785514136050, [1, 1, 1, 1, 1]), (0.4565084419100, [1, 1, 1, 1, 1]), (0.3071247857670, [1, 1, 1, 1, 1]),
    (0.2066240738900, [1, 1, 1, 1, 1]), (0.1390102977340, [1, 1, 1, 1, 1]), (0.0935218366000, [1, 1, 1, 1, 1]),
]
CU_LRI = [
    (11.608102301462, [1, 0, 0, 0, 0, 0, 0]), (8.3905970460850, [1, 0, 0, 0, 0, 0, 0]),
    (6.0649119865960, [1, 1, 0, 0, 0, 0, 0]), (4.3838545937940, [1, 1, 1, 0, 0, 0, 0]),
    (3.1687485559560, [1, 1, 1, 1, 0, 0, 0]), (2.2904426221370, [1, 1, 1, 1, 1, 0, 0]),
    (1.6555833675850, [1, 1, 1, 1, 1, 1, 0]), (1.1966928402980, [1, 1, 1, 1, 1, 1, 1]),
    (0.8649964611020, [1, 1, 1, 1, 1, 1, 1]), (0.6252388687580, [1, 1, 1, 1, 1, 1, 1]),
    (0.4519366963750, [1, 1, 1, 1, 1, 1, 1]), (0.3266699940390, [1, 1, 1, 1, 1, 1, 1]),
    (0.2361244082660, [1, 1, 1, 1, 1, 1, 1]), (0.1706760253360, [1, 1, 1, 1, 1, 1, 1]),
    (0.1233684642700, [1, 1, 1, 1, 1, 1, 1]),
]

ORBITAL = {"H-DZVP": H_DZVP, "O-DZVP": O_DZVP, "O-TZV2PX": O_TZV2PX, "Cu-DZVP": CU_DZVP}
AUX = {"H-LRI": H_LRI, "O-LRI": O_LRI, "Cu-LRI": CU_LRI}


class Sets:
    """Family-set table (host, numpy): per set a center, its K exponents and its
    contracted functions (l and K raw coefficients each, grouped by l)."""

    def __init__(self, center, nexp, exp_off, exps, nfun, fun_off, fun_l, coef_off, coefs, kind=None):
        self.center = np.asarray(center, np.float64).reshape(-1, 3)
        self.nexp = np.asarray(nexp, np.int32)
        self.exp_off = np.asarray(exp_off, np.int64)
        self.exps = np.asarray(exps, np.float64)
        self.nfun = np.asarray(nfun, np.int32)
        self.fun_off = np.asarray(fun_off, np.int64)
        self.fun_l = np.asarray(fun_l, np.int32)
        self.coef_off = np.asarray(coef_off, np.int64)
        self.coefs = np.asarray(coefs, np.float64)
        self.kind = kind

    @property
    def n(self) -> int:
        return int(self.nexp.shape[0])

    def nsgf(self) -> np.ndarray:
        """spherical functions per set: sum over its functions of 2l+1"""
        out = np.zeros(self.n, np.int64)
        for s in range(self.n):
            f0, nf = int(self.fun_off[s]), int(self.nfun[s])
            out[s] = int((2 * self.fun_l[f0:f0 + nf] + 1).sum())
        return out

    def as_shells(self):
        """every contracted function as a shell of its own (inputs.Shells) and the
        first shell of each set"""
        centers, ls, ks, exps, coefs, atom = [], [], [], [], [], []
        first = np.zeros(self.n, np.int64)
        for s in range(self.n):
            first[s] = len(ls)
            e0, k = int(self.exp_off[s]), int(self.nexp[s])
            for f in range(int(self.fun_off[s]), int(self.fun_off[s] + self.nfun[s])):
                centers.append(self.center[s])
                ls.append(int(self.fun_l[f]))
                ks.append(k)
                exps.append(self.exps[e0:e0 + k])
                coefs.append(self.coefs[self.coef_off[f]:self.coef_off[f] + k])
                atom.append(s)
        nprim = np.asarray(ks, np.int32)
        off = np.zeros(len(ks), np.int64)
        if len(ks):
            off[1:] = np.cumsum(nprim[:-1])
        sh = inputs.Shells(np.asarray(centers, np.float64).reshape(-1, 3), np.asarray(ls, np.int32), nprim, off,
                           np.concatenate(exps) if exps else np.zeros(0), np.concatenate(coefs) if coefs else
                           np.zeros(0), np.asarray(atom, np.int32))
        return sh, first


def make_sets(centers, names) -> Sets:
    """one orbital set per center, `names[i]` a key of ORBITAL"""
    nexp, exp_off, exps, nfun, fun_off, fun_l, coef_off, coefs = [], [], [], [], [], [], [], []
    for name in names:
        b = ORBITAL[name]
        k = len(b["exps"])
        exp_off.append(len(exps))
        exps.extend(b["exps"])
        nexp.append(k)
        fun_off.append(len(fun_l))
        nfun.append(len(b["l"]))
        for l, c in zip(b["l"], b["coefs"]):
            assert len(c) == k
            fun_l.append(l)
            coef_off.append(len(coefs))
            coefs.extend(c)
    return Sets(centers, nexp, exp_off, exps, nfun, fun_off, fun_l, coef_off, coefs, kind=list(names))


def aux_shells(centers, names) -> inputs.Shells:
    """LRI auxiliary functions of each center as uncontracted shells"""
    cs, ls, ex, atom = [], [], [], []
    for a, (c, name) in enumerate(zip(centers, names)):
        for e, counts in AUX[name]:
            for l, m in enumerate(counts):
                for _ in range(m):
                    cs.append(c)
                    ls.append(l)
                    ex.append(e)
                    atom.append(a)
    n = len(ls)
    return inputs.Shells(np.asarray(cs, np.float64).reshape(-1, 3), np.asarray(ls, np.int32),
                         np.ones(n, np.int32), np.arange(n, dtype=np.int64), np.asarray(ex, np.float64),
                         np.ones(n), np.asarray(atom, np.int32))
