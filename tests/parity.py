"""Parity criteria shared by the tests.

Values:      |x - y| <= 1e-12 |y| + 1e-14 max(1, max|Y|)
Derivatives: |x - y| <= 1e-10 |y| + 1e-12 max(1, max|dY|)
per element, where Y (dY) is the reference block (its three derivative blocks).
The absolute floor scales with the block's magnitude because Coulomb-type
blocks reach ~1e3 and near-zero elements arise by cancellation."""
import numpy as np

VAL_REL, VAL_ABS = 1e-12, 1e-14
DER_REL, DER_ABS = 1e-10, 1e-12


def block_ratios(x, y, off, sizes, ncomp=1, rel=VAL_REL, absf=VAL_ABS):
    """Per-block worst |x-y| / allowed (<= 1 passes)."""
    r = np.zeros(len(sizes))
    for i, (o, n) in enumerate(zip(off, sizes)):
        s = slice(ncomp * o, ncomp * o + ncomp * n)
        Y = y[s]
        X = x[s]
        sc = max(1.0, float(np.abs(Y).max())) if n else 1.0
        allowed = rel * np.abs(Y) + absf * sc
        d = np.abs(X - Y)
        if not np.all(np.isfinite(X)):
            r[i] = np.inf
        else:
            r[i] = float((d / allowed).max()) if n else 0.0
    return r


def assert_parity(x, y, off, sizes, deriv=False, what=""):
    if deriv:
        r = block_ratios(x, y, off, sizes, 3, DER_REL, DER_ABS)
    else:
        r = block_ratios(x, y, off, sizes, 1, VAL_REL, VAL_ABS)
    bad = np.nonzero(r > 1.0)[0]
    assert len(bad) == 0, f"{what}: {len(bad)} blocks outside tolerance, worst ratio {r.max():.3g} at {bad[:10]}"
    return float(r.max()) if len(r) else 0.0
