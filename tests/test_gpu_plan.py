"""Batched path (shg_plan_*): graph replay and the persistent class-binned
kernel give the same blocks as the plain per-class launches, including after
the centers change between replays."""
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


def _setup(engine, w, deriv):
    import torch
    dev = torch.device("cuda")
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.full((tot,), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((3 * tot,), float("nan"), dtype=torch.float64, device=dev) if deriv else None
    return dsh, pairs, oo, out, dout


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("op", ["coulomb", "erfc", "overlap"])
def test_plan_matches_plain(engine, persistent, op):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(77, 5000)
    print(f"case plan small5000 op={op} persistent={persistent}", flush=True)
    dsh, pairs, oo, out, dout = _setup(engine, w, True)
    engine.pairs(dsh, op, w.omega[op], pairs, oo, out, dout)
    torch.cuda.synchronize()
    ref, dref = out.clone(), dout.clone()
    out.fill_(float("nan"))
    dout.fill_(float("nan"))
    plan = shg.Plan(engine, dsh, op, w.omega[op], pairs, oo, out, dout,
                    shg.PLAN_PERSISTENT if persistent else 0)
    for rep in range(3):     # replays with eager work in between
        out.fill_(float("nan"))
        dout.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(dout, dref), f"replay {rep}"
        _ = (out * 2).sum().item()
    plan.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_plan_picks_up_new_centers(engine, persistent):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(78, 3000)
    dsh, pairs, oo, out, dout = _setup(engine, w, True)
    plan = shg.Plan(engine, dsh, "coulomb", 0.0, pairs, oo, out, dout, shg.PLAN_PERSISTENT if persistent else 0)
    # move every center; the replayed graph must see the new coordinates
    new_centers = dsh.center + torch.randn_like(dsh.center) * 0.3
    dsh.center.copy_(new_centers)
    plan.execute()
    torch.cuda.synchronize()
    got, gotd = out.clone(), dout.clone()
    out2 = torch.empty_like(out)
    dout2 = torch.empty_like(dout)
    engine.pairs(dsh, "coulomb", 0.0, pairs, oo, out2, dout2)
    torch.cuda.synchronize()
    assert torch.equal(got, out2) and torch.equal(gotd, dout2)
    plan.close()


def test_plan_autotune_selects_a_mode(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(79, 20000)
    dsh, pairs, oo, out, dout = _setup(engine, w, False)
    plan = shg.Plan(engine, dsh, "erf", w.omega["erf"], pairs, oo, out, None)
    t_cls, t_per = plan.autotune(2)
    assert t_cls > 0 and t_per > 0
    assert plan.mode == ("persistent" if t_per < t_cls else "per-class")
    assert plan.tile_order in ("heaviest-first", "alternating", "round-robin")
    plan.set_mode(True)      # the persistent kernel with the chosen tile order
    plan.execute()
    torch.cuda.synchronize()
    ref = torch.empty_like(out)
    engine.pairs(dsh, "erf", w.omega["erf"], pairs, oo, ref)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.set_mode(t_per < t_cls)
    out.fill_(float("nan"))
    plan.execute()
    torch.cuda.synchronize()
    ref = torch.empty_like(out)
    engine.pairs(dsh, "erf", w.omega["erf"], pairs, oo, ref)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()


@pytest.mark.parametrize("group", ["light", "heavy"])
@pytest.mark.parametrize("deriv", [False, True])
def test_persistent_plan_single_class_group(engine, group, deriv):
    """Persistent plans run the heavy classes (la + lb >= 5) and the light ones
    as two kernels; a pair list with only one group leaves the other launch
    empty. Every tile order gives the plain path's blocks bitwise, screened
    plans too (skipped blocks zero)."""
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(81, 6000)
    sh = w.shells
    s = sh.l[w.pairs[:, 0]] + sh.l[w.pairs[:, 1]]
    keep = s >= 5 if group == "heavy" else s <= 4
    w = inputs.Workload(f"small6000-{group}", sh, np.ascontiguousarray(w.pairs[keep]), w.ops, w.omega, True,
                        n_atoms=w.n_atoms)
    print(f"case single group {group} deriv={deriv} n={len(w.pairs)}", flush=True)
    dsh, pairs, oo, out, dout = _setup(engine, w, deriv)
    engine.pairs(dsh, "erfc", w.omega["erfc"], pairs, oo, out, dout)
    torch.cuda.synchronize()
    ref = out.clone()
    dref = dout.clone() if deriv else None
    for order in ("heaviest-first", "alternating", "round-robin"):
        plan = shg.Plan(engine, dsh, "erfc", w.omega["erfc"], pairs, oo, out, dout, shg.PLAN_PERSISTENT)
        plan.set_tile_order(order)
        out.fill_(float("nan"))
        if deriv:
            dout.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), order
        if deriv:
            assert torch.equal(dout, dref), order
        plan.close()
    plan = shg.Plan(engine, dsh, "erfc", w.omega["erfc"], pairs, oo, out, dout, shg.PLAN_PERSISTENT, tau=1e-12)
    out.fill_(float("nan"))
    plan.execute()
    torch.cuda.synchronize()
    got, r = out.cpu().numpy(), ref.cpu().numpy()
    assert np.all((got == r) | (got == 0))
    kept, _ = plan.stats()
    assert kept + len(plan.skipped()) == len(w.pairs)
    plan.close()
