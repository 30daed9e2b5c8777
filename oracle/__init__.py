"""CPU oracle for contracted SHG integrals -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It computes (a|O|b), its derivatives with
respect to R_a, (a|r_a^{2n}|b) and (a b a~) by the plain definitions (Obara-Saika recurrences
over Cartesian Gaussians, contraction, Cartesian -> real solid harmonic
transform, numerical normalisation); see ``shg_oracle.c``. It shares no code
with the GPU engine.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OPS = {"overlap": 0, "coulomb": 1, "erf": 2, "erfc": 3, "gauss": 4,
       "overlap_vrr": 5,  # overlap through the generic recurrence (self-check only)
       "gcoulomb": 6}     # exp(-w r^2)/r

_libs: dict = {}


def _lib(long_double=False):
    """long_double: False (double), True (long double) or "quad" (__float128)."""
    key = "q" if long_double == "quad" else ("ld" if long_double else "d")
    if key not in _libs:
        path = os.path.join(HERE, {"q": "liboracle_q.so", "ld": "liboracle_ld.so", "d": "liboracle.so"}[key])
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.shgo_pairs.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, C.c_double, P,
                                   C.c_int64, P, P, P]
        lib.shgo_aab.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int32, P, P, P, P, P, P, P,
                                 C.c_int64, P, P, P]
        lib.shgo_r2n.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, P, C.c_int64, P, P, P]
        lib.shgo_boys.argtypes = [C.c_int, C.c_double, P]
        lib.shgo_ss_derivs.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_int, P]
        lib.shgo_solid_harmonic.argtypes = [C.c_int, P, P]
        lib.shgo_prim_cart.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, P, P,
                                       C.c_int, C.c_int, P]
        _libs[key] = lib
    return _libs[key]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _shell_arrays(sh):
    return (np.ascontiguousarray(sh.center, np.float64), np.ascontiguousarray(sh.l, np.int32),
            np.ascontiguousarray(sh.nprim, np.int32), np.ascontiguousarray(sh.prim_off, np.int64),
            np.ascontiguousarray(sh.exps, np.float64), np.ascontiguousarray(sh.coefs, np.float64))


def num_threads() -> int:
    return int(_lib().shgo_num_threads())


def set_num_threads(n: int) -> None:
    """threads of the double-precision build's OpenMP loops (timing only)"""
    lib = _lib()
    lib.shgo_set_num_threads.argtypes = [C.c_int]
    lib.shgo_set_num_threads(int(n))


def pairs(shells, op: str, omega: float, pair_idx, out_off=None, deriv=False,
          long_double=False):
    """(a|O|b) blocks (and d/dR_a if ``deriv``) in the flat layout of the C ABI.

    Returns ``out`` (and ``dout``): block i starts at ``out_off[i]`` and is
    (2la+1)x(2lb+1) row-major, m = -l..l; ``dout`` holds the x, y, z blocks at
    ``3*out_off[i]``."""
    pair_idx = np.ascontiguousarray(pair_idx, np.int32).reshape(-1, 2)
    la = shells.l[pair_idx[:, 0]].astype(np.int64)
    lb = shells.l[pair_idx[:, 1]].astype(np.int64)
    sz = (2 * la + 1) * (2 * lb + 1)
    if out_off is None:
        out_off = np.zeros(len(sz), np.int64)
        out_off[1:] = np.cumsum(sz[:-1])
    out_off = np.ascontiguousarray(out_off, np.int64)
    total = int((out_off + sz).max()) if len(sz) else 0
    out = np.zeros(total)
    dout = np.zeros(3 * total) if deriv else None
    arrs = _shell_arrays(shells)
    rc = _lib(long_double).shgo_pairs(shells.n, *[_p(a) for a in arrs], OPS[op], float(omega),
                                      _p(pair_idx), len(pair_idx), _p(out_off), _p(out),
                                      _p(dout) if deriv else None)
    if rc != 0:
        raise ValueError(f"oracle shgo_pairs failed ({rc})")
    return (out, dout) if deriv else out


class _FunctionShells:
    """every contracted function of a family-set table as a shell of its own
    (its set's center and exponents, its own l and coefficients)"""

    def __init__(self, sets):
        centers, ls, ks, exps, coefs = [], [], [], [], []
        self.first = np.zeros(len(sets.nexp), np.int64)
        for s in range(len(sets.nexp)):
            self.first[s] = len(ls)
            e0, k = int(sets.exp_off[s]), int(sets.nexp[s])
            for f in range(int(sets.fun_off[s]), int(sets.fun_off[s] + sets.nfun[s])):
                centers.append(np.asarray(sets.center[s], np.float64))
                ls.append(int(sets.fun_l[f]))
                ks.append(k)
                exps.append(np.asarray(sets.exps[e0:e0 + k], np.float64))
                coefs.append(np.asarray(sets.coefs[int(sets.coef_off[f]):int(sets.coef_off[f]) + k], np.float64))
        self.center = np.asarray(centers, np.float64).reshape(-1, 3)
        self.l = np.asarray(ls, np.int32)
        self.nprim = np.asarray(ks, np.int32)
        self.prim_off = np.zeros(len(ks), np.int64)
        if len(ks):
            self.prim_off[1:] = np.cumsum(self.nprim[:-1])
        self.exps = np.concatenate(exps) if exps else np.zeros(0)
        self.coefs = np.concatenate(coefs) if coefs else np.zeros(0)

    @property
    def n(self):
        return int(self.l.shape[0])


def set_pairs(sets, op: str, omega: float, set_pair_idx, out_off=None, deriv=False, long_double=False):
    """Blocks of family-set pairs (Sec. III): for sets A and B with functions
    f (components m = -l..l, functions in set order) the block is the matrix of
    every function-pair integral (f_a m_a | O | f_b m_b), nsgf_a x nsgf_b
    row-major with nsgf = sum over the set's functions of 2l+1, and with
    ``deriv`` its d/dR_a blocks x, y, z at 3*out_off. By definition each entry
    is the two-center integral of two contracted functions, so it is computed
    by ``pairs`` on the functions taken as shells and placed in the block."""
    fs = _FunctionShells(sets)
    sp = np.ascontiguousarray(set_pair_idx, np.int64).reshape(-1, 2)
    nsgf = np.array([int((2 * fs.l[fs.first[s]:fs.first[s] + int(sets.nfun[s])] + 1).sum())
                     for s in range(len(sets.nexp))], np.int64)
    sz = nsgf[sp[:, 0]] * nsgf[sp[:, 1]]
    if out_off is None:
        out_off = np.zeros(len(sz), np.int64)
        out_off[1:] = np.cumsum(sz[:-1])
    total = int((out_off + sz).max()) if len(sz) else 0
    # every function pair of every set pair, then placed
    fp, where = [], []
    for i, (sa, sb) in enumerate(sp):
        ra = 0
        for fa in range(int(fs.first[sa]), int(fs.first[sa] + sets.nfun[sa])):
            na = 2 * int(fs.l[fa]) + 1
            cb = 0
            for fb in range(int(fs.first[sb]), int(fs.first[sb] + sets.nfun[sb])):
                nb = 2 * int(fs.l[fb]) + 1
                fp.append((fa, fb))
                where.append((i, ra, cb, na, nb))
                cb += nb
            ra += na
    fp = np.asarray(fp, np.int32).reshape(-1, 2)
    res = pairs(fs, op, omega, fp, deriv=deriv, long_double=long_double)
    vals, dvals = (res if deriv else (res, None))
    fsz = np.array([w[3] * w[4] for w in where], np.int64)
    foff = np.zeros(len(fsz), np.int64)
    if len(fsz):
        foff[1:] = np.cumsum(fsz[:-1])
    out = np.zeros(total)
    dout = np.zeros(3 * total) if deriv else None
    for k, (i, ra, cb, na, nb) in enumerate(where):
        ld = int(nsgf[sp[i, 1]])
        blk = int(sz[i])
        src = vals[foff[k]:foff[k] + na * nb].reshape(na, nb)
        for r in range(na):
            o = int(out_off[i]) + (ra + r) * ld + cb
            out[o:o + nb] = src[r]
        if deriv:
            for c in range(3):
                dsrc = dvals[3 * foff[k] + c * na * nb:3 * foff[k] + (c + 1) * na * nb].reshape(na, nb)
                for r in range(na):
                    o = 3 * int(out_off[i]) + c * blk + (ra + r) * ld + cb
                    dout[o:o + nb] = dsrc[r]
    return (out, dout) if deriv else out


def aab(orb, aux, triples, out_off=None, deriv=False, long_double=False):
    """(a b a~) blocks [(2la+1)][(2la~+1)][(2lb+1)] for triples (a on A, a~ on A, b on B)."""
    triples = np.ascontiguousarray(triples, np.int32).reshape(-1, 3)
    la = orb.l[triples[:, 0]].astype(np.int64)
    lt = aux.l[triples[:, 1]].astype(np.int64)
    lb = orb.l[triples[:, 2]].astype(np.int64)
    sz = (2 * la + 1) * (2 * lt + 1) * (2 * lb + 1)
    if out_off is None:
        out_off = np.zeros(len(sz), np.int64)
        out_off[1:] = np.cumsum(sz[:-1])
    out_off = np.ascontiguousarray(out_off, np.int64)
    total = int((out_off + sz).max()) if len(sz) else 0
    out = np.zeros(total)
    dout = np.zeros(3 * total) if deriv else None
    a1 = _shell_arrays(orb)
    a2 = _shell_arrays(aux)
    rc = _lib(long_double).shgo_aab(orb.n, *[_p(a) for a in a1], aux.n, *[_p(a) for a in a2],
                                    _p(triples), len(triples), _p(out_off), _p(out),
                                    _p(dout) if deriv else None)
    if rc != 0:
        raise ValueError(f"oracle shgo_aab failed ({rc})")
    return (out, dout) if deriv else out


def r2n(shells, nr: int, pair_idx, out_off=None, deriv=False, long_double=False):
    """(a|r_a^{2n}|b) blocks (Sec. II.C) and, with ``deriv``, d/dR_a (the
    operator moves with a); layout as in ``pairs``. ``long_double="quad"``
    evaluates in __float128."""
    pair_idx = np.ascontiguousarray(pair_idx, np.int32).reshape(-1, 2)
    la = shells.l[pair_idx[:, 0]].astype(np.int64)
    lb = shells.l[pair_idx[:, 1]].astype(np.int64)
    sz = (2 * la + 1) * (2 * lb + 1)
    if out_off is None:
        out_off = np.zeros(len(sz), np.int64)
        out_off[1:] = np.cumsum(sz[:-1])
    out_off = np.ascontiguousarray(out_off, np.int64)
    total = int((out_off + sz).max()) if len(sz) else 0
    out = np.zeros(total)
    dout = np.zeros(3 * total) if deriv else None
    arrs = _shell_arrays(shells)
    rc = _lib(long_double).shgo_r2n(shells.n, *[_p(a) for a in arrs], int(nr), _p(pair_idx),
                                    len(pair_idx), _p(out_off), _p(out),
                                    _p(dout) if deriv else None)
    if rc != 0:
        raise ValueError(f"oracle shgo_r2n failed ({rc})")
    return (out, dout) if deriv else out


def boys(nmax: int, T: float, long_double=False) -> np.ndarray:
    F = np.zeros(nmax + 1)
    _lib(long_double).shgo_boys(nmax, float(T), _p(F))
    return F


def ss_derivs(op: str, omega: float, a: float, b: float, R2: float, nmax: int,
              long_double=False) -> np.ndarray:
    g = np.zeros(nmax + 1)
    _lib(long_double).shgo_ss_derivs(OPS[op], omega, a, b, R2, nmax, _p(g))
    return g


def solid_harmonic(l: int):
    """(T, pw): T[(m+l), i] coefficient of Cartesian monomial pw[i] in S_lm."""
    nc = (l + 1) * (l + 2) // 2
    T = np.zeros((2 * l + 1) * nc)
    pw = np.zeros(3 * nc, np.int32)
    _lib().shgo_solid_harmonic(l, _p(T), _p(pw))
    return T.reshape(2 * l + 1, nc), pw.reshape(nc, 3)


def prim_cart(op, omega, a, b, A, B, la, lb, long_double=False):
    na, nb = (la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2
    P = np.zeros(na * nb)
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    _lib(long_double).shgo_prim_cart(OPS[op], omega, a, b, _p(A), _p(B), la, lb, _p(P))
    return P.reshape(na, nb)
