"""The CPU oracle and the host mirror (the engine's device arithmetic compiled
for the CPU) built with AddressSanitizer and UndefinedBehaviorSanitizer, every
finding fatal, and run on small cases: two-center pairs for all five operators
and exp(-w r^2)/r with d/dR_a, (a|r_a^{2n}|b) and the three-index overlap
through the oracle. Each run must exit cleanly, and its results must equal
those of the normal builds (same arithmetic, other compiler flags)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1701_06588_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(name, path):
    """a build script by path, under a module name of its own (tests/hostmirror
    has a build.py too)"""
    import importlib.util
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def exes():
    return _load("sanitize_build", os.path.join(HERE, "sanitize", "build.py")).build()


def _shells_bytes(sh):
    return b"".join([np.int32(sh.n).tobytes(), np.int64(len(sh.exps)).tobytes(),
                     np.ascontiguousarray(sh.center, np.float64).tobytes(),
                     np.ascontiguousarray(sh.l, np.int32).tobytes(), np.ascontiguousarray(sh.nprim, np.int32).tobytes(),
                     np.ascontiguousarray(sh.prim_off, np.int64).tobytes(),
                     np.ascontiguousarray(sh.exps, np.float64).tobytes(),
                     np.ascontiguousarray(sh.coefs, np.float64).tobytes()])


def _write_case(path, kind, arg, deriv, omega, shells, idx, out_off, total, aux=None):
    parts = [np.asarray([kind, arg, int(deriv)], np.int32).tobytes(), np.float64(omega).tobytes(),
             _shells_bytes(shells)]
    if aux is not None:
        parts.append(_shells_bytes(aux))
    parts += [np.int64(len(idx)).tobytes(), np.ascontiguousarray(idx, np.int32).tobytes(),
              np.ascontiguousarray(out_off, np.int64).tobytes(), np.int64(total).tobytes()]
    with open(path, "wb") as fh:
        fh.write(b"".join(parts))


def _run(exe, case, out, total, deriv):
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87")
    r = subprocess.run([exe, case, out], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"{os.path.basename(exe)} exit {r.returncode}\n{r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    v = np.fromfile(out, np.float64)
    assert v.size == total * (4 if deriv else 1)
    return v[:total], (v[total:] if deriv else None)


def _offsets(sizes):
    off = np.zeros(len(sizes), np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    return off, int(np.sum(sizes))


def _close(got, ref):
    scale = max(1.0, float(np.max(np.abs(ref)))) if ref.size else 1.0
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14 * scale), float(np.max(np.abs(got - ref)))


@pytest.mark.parametrize("op", ["overlap", "coulomb", "erf", "erfc", "gauss", "gcoulomb"])
def test_oracle_pairs_sanitized(exes, tmp_path, op):
    w = inputs.small_pairs(41, 40, lmax=4, kmax=4)
    sz = np.asarray(w.block_sizes(), np.int64)
    off, tot = _offsets(sz)
    omega = w.omega.get(op, 0.7)
    case, out = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    _write_case(case, 1, oracle.OPS[op], True, omega, w.shells, w.pairs, off, tot)
    v, d = _run(exes["oracle"], case, out, tot, True)
    rv, rd = oracle.pairs(w.shells, op, omega, w.pairs, off, deriv=True)
    _close(v, rv)
    _close(d, rd)


def test_oracle_r2n_and_aab_sanitized(exes, tmp_path):
    w = inputs.small_pairs(42, 30, lmax=3, kmax=3)
    sz = np.asarray(w.block_sizes(), np.int64)
    off, tot = _offsets(sz)
    case, out = str(tmp_path / "r2n.bin"), str(tmp_path / "r2n.out")
    _write_case(case, 2, 3, True, 0.0, w.shells, w.pairs, off, tot)
    v, d = _run(exes["oracle"], case, out, tot, True)
    rv, rd = oracle.r2n(w.shells, 3, w.pairs, off, deriv=True)
    _close(v, rv)
    _close(d, rd)
    t = inputs.small_triples(43, 24, lmax=2, ltmax=4, kmax=3)
    orb, aux, tri = t.shells, t.aux, t.triples
    tsz = ((2 * orb.l[tri[:, 0]] + 1) * (2 * aux.l[tri[:, 1]] + 1) * (2 * orb.l[tri[:, 2]] + 1)).astype(np.int64)
    toff, ttot = _offsets(tsz)
    case, out = str(tmp_path / "aab.bin"), str(tmp_path / "aab.out")
    _write_case(case, 3, 0, True, 0.0, orb, tri, toff, ttot, aux=aux)
    v, d = _run(exes["oracle"], case, out, ttot, True)
    rv, rd = oracle.aab(orb, aux, tri, toff, deriv=True)
    _close(v, rv)
    _close(d, rd)


@pytest.mark.parametrize("op", ["overlap", "coulomb", "erf", "erfc", "gauss"])
def test_host_mirror_sanitized(exes, tmp_path, op):
    import ctypes as C
    w = inputs.small_pairs(44, 60, lmax=2, kmax=7)
    sz = np.asarray(w.block_sizes(), np.int64)
    off, tot = _offsets(sz)
    case, out = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    _write_case(case, 1, oracle.OPS[op], True, w.omega[op], w.shells, w.pairs, off, tot)
    v, d = _run(exes["mirror"], case, out, tot, True)
    # the normal host-mirror build on the same case
    lib = C.CDLL(_load("hostmirror_build", os.path.join(HERE, "hostmirror", "build.py")).build())
    P = C.c_void_p
    lib.shgm_pairs.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, C.c_double, P, C.c_int64, P, P, P]
    sh = w.shells
    arr = [np.ascontiguousarray(sh.center, np.float64), np.ascontiguousarray(sh.l, np.int32),
           np.ascontiguousarray(sh.nprim, np.int32), np.ascontiguousarray(sh.prim_off, np.int64),
           np.ascontiguousarray(sh.exps, np.float64), np.ascontiguousarray(sh.coefs, np.float64)]
    pr = np.ascontiguousarray(w.pairs, np.int32)
    rv, rd = np.zeros(tot), np.zeros(3 * tot)
    rc = lib.shgm_pairs(sh.n, *[a.ctypes.data for a in arr], oracle.OPS[op], w.omega[op], pr.ctypes.data, len(pr),
                        off.ctypes.data, rv.ctypes.data, rd.ctypes.data)
    assert rc == 0
    _close(v, rv)
    _close(d, rd)
