"""GPU swap symmetry (shg_pairs_swap, Sec. V): blocks of the swapped pairs
(b, a) filled from the evaluated (a, b) blocks, against the long-double
oracle evaluated directly on the swapped pairs."""
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


@pytest.mark.parametrize("op", ["overlap", "coulomb", "erfc"])
@pytest.mark.parametrize("deriv", [False, True])
def test_swap_matches_oracle(engine, op, deriv):
    import torch
    w = inputs.small_pairs(2028, 2000)
    print(f"case swap small2000 op={op} deriv={deriv}", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    sz = w.block_sizes()
    sw = np.ascontiguousarray(w.pairs[:, ::-1], np.int32)
    # swapped blocks after the evaluated ones, in reverse pair order (ragged, non-monotone offsets)
    rev = np.arange(len(sz))[::-1]
    dst = np.zeros(len(sz), np.int64)
    dst[rev] = tot + np.concatenate([[0], np.cumsum(sz[rev][:-1])])
    out = torch.full((2 * tot,), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((6 * tot,), float("nan"), dtype=torch.float64, device=dev) if deriv else None
    p = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    engine.pairs(dsh, op, w.omega[op], p, oo, out, dout)
    engine.pairs_swap(dsh, p, oo, torch.as_tensor(dst, device=dev), out, dout, check=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    if deriv:
        ro, rd = oracle.pairs(w.shells, op, w.omega[op], sw, dst - tot, deriv=True, long_double=True)
        assert_parity(dout.cpu().numpy()[3 * tot:], rd, dst - tot, sz, True, f"swap {op} d/dR")
    else:
        ro = oracle.pairs(w.shells, op, w.omega[op], sw, dst - tot, long_double=True)
    assert_parity(o[tot:], ro, dst - tot, sz, False, f"swap {op}")
    # the transpose is exact: swapping the swapped blocks back reproduces the originals bitwise
    back = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    both = torch.cat([out[tot:], back])
    dboth = torch.cat([dout[3 * tot:], torch.zeros(3 * tot, dtype=torch.float64, device=dev)]) if deriv else None
    engine.pairs_swap(dsh, torch.as_tensor(sw, device=dev), torch.as_tensor(dst - tot, device=dev),
                      torch.as_tensor(off + tot, device=dev), both, dboth, check=True)
    torch.cuda.synchronize()
    assert np.array_equal(both.cpu().numpy()[tot:], o[:tot])
    if deriv:
        assert np.array_equal(dboth.cpu().numpy()[3 * tot:], dout.cpu().numpy()[:3 * tot])


def test_swap_errors(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(2028, 50)
    print("case swap errors", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    out = torch.zeros(2 * 81, dtype=torch.float64, device=dev)
    bad = torch.tensor([[0, w.shells.n]], dtype=torch.int32, device=dev)
    z = torch.zeros(1, dtype=torch.int64, device=dev)
    d = torch.full((1,), 81, dtype=torch.int64, device=dev)
    with pytest.raises(shg.ShgError):
        engine.pairs_swap(dsh, bad, z, d, out, check=True)
    empty = torch.zeros((0, 2), dtype=torch.int32, device=dev)
    engine.pairs_swap(dsh, empty, z[:0], d[:0], out, check=True)


def test_swap_full_five_ops500(engine):
    """The benchmark's swap configuration at full size (1.61e6 ordered pairs,
    Coulomb, values + d/dR_a): plan over the pairs with a <= b, the mirror
    blocks by shg_pairs_swap, every element against the plain evaluation of all
    pairs (1e-12 relative, 1e-14 of the largest element as floor)."""
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.five_ops500()
    print(f"case swap five_ops500 pairs={len(w.pairs)}", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    n = len(w.pairs)
    a_, b_ = w.pairs[:, 0].astype(np.int64), w.pairs[:, 1].astype(np.int64)
    key = a_ * int(w.shells.n) + b_
    kord = np.argsort(key)
    mir = np.nonzero(a_ > b_)[0]
    partner = kord[np.searchsorted(key[kord], b_[mir] * int(w.shells.n) + a_[mir])]
    assert np.all(key[partner] == b_[mir] * int(w.shells.n) + a_[mir])
    ci = np.nonzero(a_ <= b_)[0]
    ref = torch.empty(tot, dtype=torch.float64, device=dev)
    dref = torch.empty(3 * tot, dtype=torch.float64, device=dev)
    engine.pairs(dsh, "coulomb", 0.0, torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev),
                 torch.as_tensor(off, device=dev), ref, dref)
    out = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((3 * tot,), float("nan"), dtype=torch.float64, device=dev)
    plan = shg.Plan(engine, dsh, "coulomb", 0.0, torch.as_tensor(np.ascontiguousarray(w.pairs[ci], np.int32), device=dev),
                    torch.as_tensor(off[ci], device=dev), out, dout, flags=1)
    plan.execute()
    engine.pairs_swap(dsh, torch.as_tensor(np.ascontiguousarray(w.pairs[partner], np.int32), device=dev),
                      torch.as_tensor(off[partner], device=dev), torch.as_tensor(off[mir], device=dev), out, dout,
                      check=True)
    torch.cuda.synchronize()
    plan.close()
    for x, r, what in ((out, ref, "values"), (dout, dref, "d/dR_a")):
        assert bool(torch.isfinite(x).all().item()), what
        tol = 1e-12 * r.abs() + 1e-14 * max(1.0, r.abs().max().item())
        assert int(((x - r).abs() > tol).sum().item()) == 0, what
