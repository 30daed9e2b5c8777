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


def _assert_close_blockwise(got, ref, starts, sizes, what):
    """|got - ref| <= 64 eps max|ref block| per element: the fused kernel forms the
    same sums as the single-operator path, but the compiler may contract a
    multiply-add into an FMA in one kernel and not in the other."""
    bmax = np.maximum.reduceat(np.abs(ref), starts)
    scale = np.repeat(bmax, sizes)
    err = np.abs(got - ref)
    assert np.all(err <= 64 * np.finfo(np.float64).eps * scale), (what, float((err / np.maximum(scale, 1e-300)).max()))


@pytest.mark.parametrize("deriv", [False, True])
@pytest.mark.parametrize("ops", [("overlap", "coulomb", "erfc", "erf", "gauss"), ("erfc", "coulomb")])
def test_multi_plan_matches_single_operator_path(engine, deriv, ops):
    """One kernel for several operators gives each operator's blocks of the
    single-operator path (values bitwise where both kernels round alike; every
    element within 64 eps of its block's largest element)."""
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.small_pairs(79, 4000)
    print(f"case multi plan small4000 ops={ops} deriv={deriv}", flush=True)
    dsh, pairs, oo, out, dout = _setup(engine, w, deriv)
    refs = []
    for op in ops:
        engine.pairs(dsh, op, w.omega[op], pairs, oo, out, dout)
        torch.cuda.synchronize()
        refs.append((out.clone(), dout.clone() if deriv else None))
    outs = [torch.full_like(out, float("nan")) for _ in ops]
    douts = [torch.full_like(dout, float("nan")) for _ in ops] if deriv else None
    plan = shg.MultiPlan(engine, dsh, ops, [w.omega[o] for o in ops], pairs, oo, outs, douts)
    assert plan.mode == "multi" and plan.n_skipped == 0
    for rep in range(2):
        for k in range(len(ops)):
            outs[k].fill_(float("nan"))
            if deriv:
                douts[k].fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        off, tot = w.out_offsets()
        sz = np.asarray(w.block_sizes(), np.int64)
        for k, op in enumerate(ops):
            _assert_close_blockwise(outs[k].cpu().numpy(), refs[k][0].cpu().numpy(), off, sz, (op, rep))
            if deriv:
                _assert_close_blockwise(douts[k].cpu().numpy(), refs[k][1].cpu().numpy(), 3 * off, 3 * sz,
                                        (op, rep, "deriv"))
    kept, nbytes = plan.stats()
    assert kept == len(w.pairs)
    plan.close()


def test_multi_plan_screened(engine):
    import torch
    from paper_1701_06588_amd import shg
    w = inputs.screen5000(n_atoms=700, box=24.0)
    ops = ("overlap", "gauss", "coulomb")
    print(f"case multi plan screened n={len(w.pairs)}", flush=True)
    dsh, pairs, oo, out, dout = _setup(engine, w, True)
    refs = []
    for op in ops:
        engine.pairs(dsh, op, w.omega[op], pairs, oo, out, dout)
        torch.cuda.synchronize()
        refs.append((out.cpu().numpy(), dout.cpu().numpy()))
    outs = [torch.full_like(out, float("nan")) for _ in ops]
    douts = [torch.full_like(dout, float("nan")) for _ in ops]
    tau = 1e-12
    plan = shg.MultiPlan(engine, dsh, ops, [w.omega[o] for o in ops], pairs, oo, outs, douts, tau=tau)
    plan.execute()
    torch.cuda.synchronize()
    skipped = np.zeros(len(w.pairs), bool)
    skipped[plan.skipped()] = True
    assert skipped.sum() == plan.n_skipped > 0
    off, tot = w.out_offsets()
    sz = np.asarray(w.block_sizes(), np.int64)
    es, ds = np.repeat(skipped, sz), np.repeat(skipped, 3 * sz)
    for k, op in enumerate(ops):
        g, dg = outs[k].cpu().numpy(), douts[k].cpu().numpy()
        r, dr = refs[k]
        gz, dgz = g.copy(), dg.copy()
        gz[es] = r[es]
        dgz[ds] = dr[ds]
        _assert_close_blockwise(gz, r, off, sz, op)
        _assert_close_blockwise(dgz, dr, 3 * off, 3 * sz, (op, "deriv"))
        assert np.all(g[es] == 0) and np.all(dg[ds] == 0), op
        # skipped only when every operator's bound is below tau, so every skipped element is tiny
        assert np.all(np.abs(r[es]) <= tau) and np.all(np.abs(dr[ds]) <= tau), op
    plan.close()
