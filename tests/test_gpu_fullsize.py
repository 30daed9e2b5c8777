"""Full-size workloads in the launch configuration the benchmark times, checked
against the long-double oracle on sampled blocks: the 256 uneven molecules
through a persistent plan (values and d/dR_a), and the 5000-atom screening
workload (Coulomb and erfc values) through a screened plan whose skipped
blocks must be tiny in the exact result."""
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


def _gather(buf, off, sz, idx, ncomp):
    """the blocks `idx` of a device buffer, concatenated on the host"""
    import torch
    pos = np.concatenate([np.arange(ncomp * off[i], ncomp * (off[i] + sz[i])) for i in idx])
    return buf[torch.as_tensor(pos, device=buf.device)].cpu().numpy()


def _sub_offsets(sz, idx):
    o = np.zeros(len(idx), np.int64)
    o[1:] = np.cumsum(sz[idx][:-1])
    return o


def test_molecules256_persistent_plan_sampled(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.molecules256()
    op = "erfc"
    print(f"case molecules256 op={op} n={len(w.pairs)}", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    sz = np.asarray(w.block_sizes(), np.int64)
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((3 * tot,), float("nan"), dtype=torch.float64, device=dev)
    plan = shg.Plan(engine, dsh, op, w.omega[op], pairs, oo, out, dout, shg.PLAN_PERSISTENT)
    out.fill_(float("nan"))
    dout.fill_(float("nan"))
    plan.execute()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all()) and bool(torch.isfinite(dout).all())
    idx = np.sort(np.random.default_rng(11).choice(len(w.pairs), 1500, replace=False))
    so = _sub_offsets(sz, idx)
    ro, rd = oracle.pairs(w.shells, op, w.omega[op], w.pairs[idx], so, deriv=True, long_double=True)
    assert_parity(_gather(out, off, sz, idx, 1), ro, so, sz[idx], False, "molecules256")
    assert_parity(_gather(dout, off, sz, idx, 3), rd, so, sz[idx], True, "molecules256 deriv")
    plan.close()


@pytest.mark.parametrize("op", ["coulomb", "erfc"])
def test_screen5000_screened_plan_sampled(engine, op):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.screen5000()
    print(f"case screen5000 op={op} n={len(w.pairs)}", flush=True)
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    sz = np.asarray(w.block_sizes(), np.int64)
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    tau = 1e-10 / (2 * len(w.pairs))
    plan = shg.Plan(engine, dsh, op, w.omega[op], pairs, oo, out, None, shg.PLAN_PERSISTENT, tau=tau)
    plan.execute()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    skipped = plan.skipped()
    rng = np.random.default_rng(12)
    kept = np.setdiff1d(np.arange(len(w.pairs)), skipped)
    idx = np.sort(rng.choice(kept, 1500, replace=False))
    so = _sub_offsets(sz, idx)
    ro = oracle.pairs(w.shells, op, w.omega[op], w.pairs[idx], so, long_double=True)
    assert_parity(_gather(out, off, sz, idx, 1), ro, so, sz[idx], False, "screen5000 kept")
    if len(skipped):
        sk = np.sort(rng.choice(skipped, min(500, len(skipped)), replace=False))
        sso = _sub_offsets(sz, sk)
        assert np.all(_gather(out, off, sz, sk, 1) == 0.0)
        # every skipped block of the plain GPU path is below tau
        ref = torch.empty_like(out)
        engine.pairs(dsh, op, w.omega[op], pairs, oo, ref)
        torch.cuda.synchronize()
        assert np.all(np.abs(_gather(ref, off, sz, skipped, 1)) <= tau)
        # and so is the oracle's, except on same-center pairs with la != lb: those
        # blocks are exactly zero, and the oracle's Cartesian route leaves
        # rounding noise there
        la = w.shells.l[w.pairs[sk, 0]]
        lb = w.shells.l[w.pairs[sk, 1]]
        same = np.all(w.shells.center[w.pairs[sk, 0]] == w.shells.center[w.pairs[sk, 1]], axis=1)
        exact_zero = same & (la != lb)
        rs = oracle.pairs(w.shells, op, w.omega[op], w.pairs[sk], sso, long_double=True)
        blk = np.repeat(exact_zero, sz[sk])
        assert np.all(np.abs(rs[~blk]) <= tau)
    plan.close()
