"""The engine's FP64 device arithmetic (csrc/shg_math.h), compiled for the CPU,
against the long-double oracle: every (la, lb) class, all five operators,
values and d/dR_a. Catches formula errors without a GPU."""
import ctypes as C
import os
import sys

import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1701_06588_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "hostmirror"))


@pytest.fixture(scope="module")
def hm():
    import build as hm_build
    lib = C.CDLL(hm_build.build())
    P = C.c_void_p
    lib.shgm_pairs.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, C.c_double, P, C.c_int64, P, P, P]
    lib.shgm_boys.argtypes = [C.c_int, C.c_double, P]
    lib.shgm_r2n.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, P, C.c_int64, P, P, P]
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def run_hm(lib, w, op):
    sh = w.shells
    off, tot = w.out_offsets()
    out, dout = np.zeros(tot), np.zeros(3 * tot)
    rc = lib.shgm_pairs(sh.n, _p(sh.center), _p(sh.l), _p(sh.nprim), _p(sh.prim_off), _p(sh.exps),
                        _p(sh.coefs), oracle.OPS[op], w.omega[op], _p(np.ascontiguousarray(w.pairs)),
                        len(w.pairs), _p(off), _p(out), _p(dout))
    assert rc == 0
    return out, dout


@pytest.mark.parametrize("op", ["overlap", "coulomb", "erf", "erfc", "gauss"])
def test_host_mirror_vs_oracle(hm, op):
    w = inputs.small_pairs(5, 300, lmax=4, kmax=7)
    off, _ = w.out_offsets()
    sz = w.block_sizes()
    out, dout = run_hm(hm, w, op)
    ro, rd = oracle.pairs(w.shells, op, w.omega[op], w.pairs, off, deriv=True, long_double=True)
    assert_parity(out, ro, off, sz, False, op)
    assert_parity(dout, rd, off, sz, True, op)


def test_host_mirror_boys_vs_mpmath(hm):
    import mpmath
    mpmath.mp.dps = 40
    worst = 0.0
    for T in [0.0, 1e-9, 0.013, 0.5, 1.03125, 2.7, 9.99, 17.3, 29.0, 35.97, 36.0, 36.5, 50.0, 300.0, 3000.0]:
        F = np.zeros(10)
        hm.shgm_boys(9, T, _p(F))
        for n in range(10):
            ref = (mpmath.mpf(1) / (2 * n + 1) if T == 0 else
                   mpmath.gammainc(n + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (n + 0.5)))
            worst = max(worst, abs(F[n] - float(ref)) / float(ref))
    assert worst < 2e-14, worst


@pytest.mark.parametrize("nr", [0, 1, 2, 3, 4, 5])
def test_host_mirror_r2n_vs_oracle(hm, nr):
    """(a|r_a^{2n}|b): the engine's double-double monopole T^(k) and block
    assembly on the CPU against the __float128 oracle, every (la, lb) class."""
    w = inputs.small_pairs(2026, 800)
    sh = w.shells
    off, tot = w.out_offsets()
    sz = w.block_sizes()
    out, dout = np.zeros(tot), np.zeros(3 * tot)
    rc = hm.shgm_r2n(sh.n, _p(sh.center), _p(sh.l), _p(sh.nprim), _p(sh.prim_off), _p(sh.exps), _p(sh.coefs),
                     nr, _p(np.ascontiguousarray(w.pairs)), len(w.pairs), _p(off), _p(out), _p(dout))
    assert rc == 0
    ro, rd = oracle.r2n(sh, nr, w.pairs, off, deriv=True, long_double="quad")
    assert_parity(out, ro, off, sz, False, f"r2n n={nr}")
    assert_parity(dout, rd, off, sz, True, f"r2n n={nr} d/dR_a")
