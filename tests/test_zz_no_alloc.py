"""shg_pairs_noalloc (fixed library scratch, no allocation in the call) against
shg_pairs_deriv / shg_pairs on the same inputs: two calls in a row, the second
with a smaller input, every block bitwise equal (same kernels and tile shapes);
inputs beyond the scratch limits are rejected on the host."""
import numpy as np
import pytest

from paper_1701_06588_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    from paper_1701_06588_amd import shg
    e = shg.Engine()
    yield e
    e.close()


def _upload(engine, w):
    import torch
    dev = torch.device("cuda")
    off, tot = w.out_offsets()
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    return engine.shells(w.shells), pairs, torch.as_tensor(off, device=dev), tot


def _both(engine, w, op, deriv):
    import torch
    dsh, pairs, oo, tot = _upload(engine, w)
    dev = pairs.device
    mk = lambda k: torch.full((max(k * tot, 1),), float("nan"), dtype=torch.float64, device=dev)
    ref, got = mk(1), mk(1)
    dref, dgot = (mk(3), mk(3)) if deriv else (None, None)
    engine.pairs(dsh, op, w.omega[op], pairs, oo, ref, dref)
    engine.pairs_noalloc(dsh, op, w.omega[op], pairs, oo, got, dgot)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(got[:tot]).all())
    assert torch.equal(got[:tot], ref[:tot])
    if deriv:
        assert torch.equal(dgot[:3 * tot], dref[:3 * tot])


@pytest.mark.parametrize("op,deriv", [("coulomb", True), ("erfc", False)])
def test_noalloc_matches_plain_twice_shrinking(engine, op, deriv):
    big = inputs.small_pairs(777, 3000)
    small = inputs.small_pairs(778, 257)
    print(f"case noalloc op={op} deriv={deriv} n=3000 then 257", flush=True)
    _both(engine, big, op, deriv)
    _both(engine, small, op, deriv)


def test_noalloc_workload_share(engine):
    """a 64k-pair slice of the 500-atom workload (all classes, ragged tiles)"""
    w = inputs.five_ops500()
    sub = inputs.Workload("five_ops500[:65536]", w.shells, w.pairs[:65536], w.ops, w.omega, True)
    print("case noalloc five_ops500[:65536] gauss deriv", flush=True)
    _both(engine, sub, "gauss", True)


def test_noalloc_limits(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(5, 4)
    dsh, pairs, oo, tot = _upload(engine, w)
    out = torch.zeros(tot, dtype=torch.float64, device=pairs.device)
    big = torch.zeros((shg.NOALLOC_MAX_PAIRS + 1, 2), dtype=torch.int32, device=pairs.device)
    big_off = torch.zeros(shg.NOALLOC_MAX_PAIRS + 1, dtype=torch.int64, device=pairs.device)
    with pytest.raises(shg.ShgError):
        engine.pairs_noalloc(dsh, "overlap", 0.0, big, big_off, out)
    with pytest.raises(shg.ShgError):
        engine.pairs_noalloc(dsh, "gcoulomb", 0.7, pairs, oo, out)
    engine.pairs_noalloc(dsh, "overlap", 0.0, pairs[:0], oo[:0], out)   # n = 0: no-op
