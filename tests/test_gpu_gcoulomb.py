"""GPU parity of the Gaussian-damped Coulomb operator exp(-omega r^2)/r
(Table S1) through shg_pairs / shg_pairs_deriv against the long-double CPU
oracle, element by element."""
import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1701_06588_amd import inputs

pytestmark = pytest.mark.gpu
OMEGA = 0.7


@pytest.fixture(scope="module")
def engine():
    from paper_1701_06588_amd import shg
    e = shg.Engine()
    yield e
    e.close()


def run_gc(engine, w, deriv, omega=OMEGA, pairs=None):
    import torch
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    pr = w.pairs if pairs is None else pairs
    la = w.shells.l[pr[:, 0]].astype(np.int64)
    lb = w.shells.l[pr[:, 1]].astype(np.int64)
    sz = (2 * la + 1) * (2 * lb + 1)
    off = np.zeros(len(sz), np.int64)
    off[1:] = np.cumsum(sz[:-1])
    tot = int(sz.sum())
    p = torch.as_tensor(np.ascontiguousarray(pr, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((max(tot, 1),), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((max(3 * tot, 1),), float("nan"), dtype=torch.float64, device=dev) if deriv else None
    engine.pairs(dsh, "gcoulomb", omega, p, oo, out, dout)
    torch.cuda.synchronize()
    return off, sz, out.cpu().numpy()[:tot], (dout.cpu().numpy()[:3 * tot] if deriv else None)


@pytest.mark.parametrize("deriv", [False, True])
@pytest.mark.parametrize("omega", [0.05, OMEGA, 20.0])
def test_gcoulomb_all_classes_random(engine, deriv, omega):
    """2500 random pairs: every (la, lb) class with l <= 4, K in 1..7,
    exponents [0.05, 50], 10% same-center; several tiles per class."""
    w = inputs.small_pairs(2027, 2500)
    print(f"case gcoulomb small2500 omega={omega} deriv={deriv}", flush=True)
    off, sz, out, dout = run_gc(engine, w, deriv, omega)
    if deriv:
        ro, rd = oracle.pairs(w.shells, "gcoulomb", omega, w.pairs, off, deriv=True, long_double=True)
        assert_parity(dout, rd, off, sz, True, "gcoulomb d/dR_a")
    else:
        ro = oracle.pairs(w.shells, "gcoulomb", omega, w.pairs, off, long_double=True)
    assert_parity(out, ro, off, sz, False, "gcoulomb")


def test_gcoulomb_errors_and_plans(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(2027, 300)
    print("case gcoulomb errors", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    p = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    off, tot = w.out_offsets()
    oo = torch.as_tensor(off, device=dev)
    out = torch.zeros(tot, dtype=torch.float64, device=dev)
    for bad in (0.0, -1.0, float("inf")):
        with pytest.raises(shg.ShgError):
            engine.pairs(dsh, "gcoulomb", bad, p, oo, out)
    with pytest.raises(shg.ShgError):   # screening has no bound for this operator
        shg.Plan(engine, dsh, "gcoulomb", OMEGA, p, oo, out, tau=1e-12)
    # the context stays usable
    a = run_gc(engine, w, False)
    b = run_gc(engine, w, False)
    assert np.array_equal(a[2], b[2])


def test_gcoulomb_full_five_ops500_sampled(engine):
    """The full 500-atom pair list (~1.6e6 pairs, values + d/dR_a) in one call;
    1500 sampled blocks against the oracle."""
    w = inputs.five_ops500()
    print(f"case gcoulomb five_ops500 pairs={len(w.pairs)}", flush=True)
    off, sz, out, dout = run_gc(engine, w, True)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(dout))
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(len(w.pairs), 1500, replace=False))
    sub_off = np.zeros(len(idx), np.int64)
    sub_off[1:] = np.cumsum(sz[idx][:-1])
    ro, rd = oracle.pairs(w.shells, "gcoulomb", OMEGA, w.pairs[idx], sub_off, deriv=True, long_double=True)
    got = np.concatenate([out[off[i]:off[i] + sz[i]] for i in idx])
    gotd = np.concatenate([dout[3 * off[i]:3 * off[i] + 3 * sz[i]] for i in idx])
    assert_parity(got, ro, sub_off, sz[idx], False, "gcoulomb five_ops500")
    assert_parity(gotd, rd, sub_off, sz[idx], True, "gcoulomb five_ops500 d/dR_a")


@pytest.mark.parametrize("flags", [0, 1])
def test_gcoulomb_plan_matches_plain(engine, flags):
    """Plans (radial stage and precomputed-monopole tiles in one graph; per-class
    launches or the persistent kernel) against the plain path, replayed twice
    with the library's own work in between, then autotuned."""
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(2027, 2500)
    print(f"case gcoulomb plan flags={flags}", flush=True)
    off, sz, ref, dref = run_gc(engine, w, True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    p = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((len(ref),), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((len(dref),), float("nan"), dtype=torch.float64, device=dev)
    plan = shg.Plan(engine, dsh, "gcoulomb", OMEGA, p, oo, out, dout, flags=flags)
    for rep in range(2):
        out.fill_(float("nan"))
        dout.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        assert_parity(out.cpu().numpy(), ref, off, sz, False, f"plan rep {rep}")
        assert_parity(dout.cpu().numpy(), dref, off, sz, True, f"plan rep {rep} d/dR_a")
        run_gc(engine, w, False)     # other work on the library between replays
    plan.autotune(2)
    out.fill_(float("nan"))
    plan.execute()
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), ref, off, sz, False, f"plan autotuned ({plan.mode})")
    plan.close()
