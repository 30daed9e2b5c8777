"""Algorithmic work model of the SHG hot path (bytes and element counts).

Bytes per shell-pair block (the unit of the throughput metric):
    B(la, lb, D) = 8 (2la+1)(2lb+1)(1 + 3D)   output values (+ d/dR_a x, y, z)
                 + 8                           pair indices (2 x int32)
                 + 8                           output offset (int64)
The basis itself (centers, exponents, coefficients) is read once and is
negligible. Per (a b a~) triple the output is 8 (2la+1)(2la~+1)(2lb+1)(1+3D)
plus 12 + 8 bytes of indices and offset.

Floating-point operations per shell-pair block (add and multiply 1, FMA 2;
exp, sqrt, divisions and Boys-table reads are not converted into flops), for
primitive pairs P = Ka Kb, n_k = min(la, lb) + 1 + D radial orders and
m = min(la, lb):
    radial       P (8 + c_op (la + lb + D + 1))   c_op: overlap and Gaussian 2,
                                                  1/r and erf 6, erfc 12
    contraction  2 P n_k                           (eq. O_rab2_deriv)
    angular      24 (la+1)(lb+1) S + 2 (2la+1)(2lb+1) S,  S = (m+1)(m+2)/2
    assembly     2 (2la+1)(2lb+1)(m+1)             (eq. final_r12int_ab)
                 + 36 (2la+1)(2lb+1)(m+1) with D   (eq. dev_ab and the
                                                   derivative recurrences of Qtilde)

Contraction counts (Table 2 of the paper): the number of contracted matrix
elements for one family basis set on both centers,
    Obara-Saika:  (K * sum over the distinct l of (2l+1))^2  * (1 or 4)
    SHG:          K^2 * (2 l_max + 1 + D)
(the SHG implementation of the paper contracts k = 0..2 l_max (+1), more scalar
derivatives than strictly needed, so that the contraction is one matrix product).
"""
from __future__ import annotations

import numpy as np


def pair_bytes(la, lb, deriv: bool):
    la = np.asarray(la, dtype=np.int64)
    lb = np.asarray(lb, dtype=np.int64)
    return 8 * (2 * la + 1) * (2 * lb + 1) * (4 if deriv else 1) + 16


def triple_bytes(la, lt, lb, deriv: bool):
    la, lt, lb = (np.asarray(x, dtype=np.int64) for x in (la, lt, lb))
    return 8 * (2 * la + 1) * (2 * lt + 1) * (2 * lb + 1) * (4 if deriv else 1) + 20


C_OP = {"overlap": 2, "gauss": 2, "coulomb": 6, "erf": 6, "erfc": 12}


def pair_flops(la, lb, ka, kb, op: str, deriv: bool):
    la, lb, ka, kb = (np.asarray(x, dtype=np.int64) for x in (la, lb, ka, kb))
    d = 1 if deriv else 0
    m = np.minimum(la, lb)
    P = ka * kb
    S = (m + 1) * (m + 2) // 2
    nel = (2 * la + 1) * (2 * lb + 1)
    radial = P * (8 + C_OP[op] * (la + lb + d + 1))
    contraction = 2 * P * (m + 1 + d)
    angular = 24 * (la + 1) * (lb + 1) * S + 2 * nel * S
    assembly = 2 * nel * (m + 1) + (36 * nel * (m + 1) if deriv else 0)
    return radial + contraction + angular + assembly


def workload_flops(w, op: str, deriv: bool, mask=None) -> int:
    a, b = w.pairs[:, 0], w.pairs[:, 1]
    f = pair_flops(w.shells.l[a], w.shells.l[b], w.shells.nprim[a], w.shells.nprim[b], op, deriv)
    return int(f.sum() if mask is None else f[mask].sum())


def workload_bytes(w, deriv: bool) -> int:
    la = w.shells.l[w.pairs[:, 0]]
    lb = w.shells.l[w.pairs[:, 1]]
    return int(pair_bytes(la, lb, deriv).sum())


def contraction_counts(K: int, shell_ls, deriv: bool) -> tuple[int, int]:
    """(OS, SHG) contracted matrix elements for a family basis with contraction
    length K and shells of angular momenta `shell_ls` on both centers."""
    distinct = sorted(set(int(l) for l in shell_ls))
    os_count = (K * sum(2 * l + 1 for l in distinct)) ** 2 * (4 if deriv else 1)
    shg_count = K * K * (2 * max(distinct) + 1 + (1 if deriv else 0))
    return os_count, shg_count
