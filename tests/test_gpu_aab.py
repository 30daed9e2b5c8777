"""GPU parity of shg_aab (three-index overlap and d/dR_A) against the
long-double oracle, every (la, la~, lb) class with la, lb <= 3, la~ <= 6."""
import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1701_06588_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    from paper_1701_06588_amd import shg
    e = shg.Engine()
    yield e
    e.close()


def run_aab(engine, w, deriv):
    import torch
    dev = torch.device("cuda")
    orb = engine.shells(w.shells)
    aux = engine.shells(w.aux)
    off, tot = w.out_offsets()
    tri = torch.as_tensor(np.ascontiguousarray(w.triples, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((max(tot, 1),), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((max(3 * tot, 1),), float("nan"), dtype=torch.float64, device=dev) if deriv else None
    engine.aab(orb, aux, tri, oo, out, dout)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:tot], (dout.cpu().numpy()[:3 * tot] if deriv else None)


@pytest.mark.parametrize("deriv", [False, True])
def test_aab_random_triples(engine, deriv):
    w = inputs.small_triples(2025, 1200)
    print(f"case smalltri1200 deriv={deriv}", flush=True)
    off, _ = w.out_offsets()
    sz = w.block_sizes()
    out, dout = run_aab(engine, w, deriv)
    if deriv:
        ro, rd = oracle.aab(w.shells, w.aux, w.triples, off, deriv=True, long_double=True)
        assert_parity(dout, rd, off, sz, True, "aab deriv")
    else:
        ro = oracle.aab(w.shells, w.aux, w.triples, off, long_double=True)
    assert_parity(out, ro, off, sz, False, "aab")


def test_aab_workload_sample(engine):
    """The 2000-atom RI workload restricted to 300 atom pairs (33,600 triples),
    sampled blocks against the oracle."""
    full = inputs.aab2000()
    sel = np.arange(0, 300 * 112)
    w = inputs.Workload("aab_sub", full.shells, full.pairs, full.ops, {}, True, aux=full.aux,
                        triples=full.triples[sel])
    print(f"case aab2000[:{len(sel)}]", flush=True)
    off, _ = w.out_offsets()
    sz = w.block_sizes()
    out, dout = run_aab(engine, w, True)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(dout))
    idx = np.sort(np.random.default_rng(3).choice(len(sel), 600, replace=False))
    sub_off = np.zeros(len(idx), np.int64)
    sub_off[1:] = np.cumsum(sz[idx][:-1])
    ro, rd = oracle.aab(w.shells, w.aux, w.triples[idx], sub_off, deriv=True, long_double=True)
    got = np.concatenate([out[off[i]:off[i] + sz[i]] for i in idx])
    gotd = np.concatenate([dout[3 * off[i]:3 * off[i] + 3 * sz[i]] for i in idx])
    assert_parity(got, ro, sub_off, sz[idx], False, "aab2000 sample")
    assert_parity(gotd, rd, sub_off, sz[idx], True, "aab2000 sample deriv")


def test_aab_errors(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_triples(5, 10)
    dev = torch.device("cuda")
    off, tot = w.out_offsets()
    orb, aux = engine.shells(w.shells), engine.shells(w.aux)
    out = torch.zeros(tot, dtype=torch.float64, device=dev)
    tri = w.triples.copy()
    tri[0, 1] = 1          # a~ on a different center than a
    with pytest.raises(shg.ShgError):
        engine.aab(orb, aux, torch.as_tensor(tri, device=dev), torch.as_tensor(off, device=dev), out)
    engine.aab(orb, aux, torch.as_tensor(w.triples, device=dev), torch.as_tensor(off, device=dev), out)


@pytest.mark.parametrize("chunk", [37, 500])
def test_aab_multichunk(engine, chunk):
    """Small work items: every class of 1200 random triples spans several chunks
    (second and later chunks use their own offsets into the radial and block
    scratch) spread over the four streams; every value and d/dR_A block
    against the long-double oracle."""
    w = inputs.small_triples(4242, 1200)
    print(f"case smalltri1200 chunk={chunk}", flush=True)
    off, _ = w.out_offsets()
    sz = w.block_sizes()
    engine.set_aab_chunk(chunk)
    try:
        out, dout = run_aab(engine, w, True)
    finally:
        engine.set_aab_chunk(1 << 17)
    ro, rd = oracle.aab(w.shells, w.aux, w.triples, off, deriv=True, long_double=True)
    assert_parity(out, ro, off, sz, False, f"aab chunk {chunk}")
    assert_parity(dout, rd, off, sz, True, f"aab chunk {chunk} deriv")


def test_aab_chunk_bounds(engine):
    from paper_1701_06588_amd import shg
    for bad in (0, -1, (1 << 24) + 1):
        with pytest.raises(shg.ShgError):
            engine.set_aab_chunk(bad)


def test_aab2000_fullsize_sampled(engine):
    """The full 2000-atom RI workload in one call with the default work items
    (2^17 triples; every one of its 112 classes has about 1.9e5 triples, so
    each takes two chunks and about a third of the triples sit in a second
    chunk): values and d/dR_A of all ~2.15e7 triples (77 GB), all finite, and
    800 sampled triples against the long-double oracle."""
    import torch
    w = inputs.aab2000()
    n = len(w.triples)
    print(f"case aab2000 full n={n}", flush=True)
    dev = torch.device("cuda")
    off, tot = w.out_offsets()
    sz = np.asarray(w.block_sizes(), np.int64)
    orb, aux = engine.shells(w.shells), engine.shells(w.aux)
    tri = torch.as_tensor(np.ascontiguousarray(w.triples, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((3 * tot,), float("nan"), dtype=torch.float64, device=dev)
    engine.aab(orb, aux, tri, oo, out, dout)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all()) and bool(torch.isfinite(dout).all())
    idx = np.sort(np.random.default_rng(31).choice(n, 800, replace=False))
    so = np.zeros(len(idx), np.int64)
    so[1:] = np.cumsum(sz[idx][:-1])
    pos = torch.as_tensor(np.concatenate([np.arange(off[i], off[i] + sz[i]) for i in idx]), device=dev)
    dpos = torch.as_tensor(np.concatenate([np.arange(3 * off[i], 3 * off[i] + 3 * sz[i]) for i in idx]), device=dev)
    got, gotd = out[pos].cpu().numpy(), dout[dpos].cpu().numpy()
    del out, dout
    torch.cuda.empty_cache()
    ro, rd = oracle.aab(w.shells, w.aux, w.triples[idx], so, deriv=True, long_double=True)
    assert_parity(got, ro, so, sz[idx], False, "aab2000 full")
    assert_parity(gotd, rd, so, sz[idx], True, "aab2000 full deriv")
