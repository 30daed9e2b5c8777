"""Benchmark: contracted shell-pair blocks per second on one MI355X.

Workload (one "step"): the 500-atom system in a 20 bohr cube, 4 shells per atom
(l 0..4, K 1..7, exponents log-uniform [0.05, 50]), every ordered atom pair
within 12 bohr (1.61e6 shell pairs), evaluated for all five operators (overlap,
Coulomb, erfc(0.11 r)/r, erf(0.33 r)/r, exp(-r^2)) with values and d/dR_a.
Inputs are synthetic (seeded) and resident in HBM before the timed region.

Four paths over the same pair lists, each timed with HIP events on the
library stream over --steps steps after --warmup untimed ones:
  plain             shg_pairs_deriv per operator (binning + one launch per class)
  batched           one recorded plan per operator (binned once, hipGraph replay,
                    persistent or per-class launch chosen by the plan autotuner)
  batched+screened  the same with screening: pairs whose analytic bound (covering
                    values and d/dR_a) is below tau_blk = 1e-10 / N_candidates are
                    skipped (blocks zeroed once when the plan is made)
  batched+screened+swap  screened plans over the pairs with a <= b only; the
                    (b, a) blocks are filled by shg_pairs_swap (transpose, and
                    minus the transpose for d/dR, Sec. V); audited element-wise
                    against the plain path
`value` is the batched+screened rate in candidate blocks per second (every
block of the step counts, skipped or not). Kept blocks are checked bitwise
against the plain path; the missed mass is exact (L1 of the plain path's values
and derivatives over every skipped block).

Prints ONE JSON line. Fields beyond the common contract:
  roofline      dominant kernel of the value path, measured live with HIP events
                on the library stream: algorithmic bytes (and flops) per launch
                from workmodel.py over the pairs the launch evaluates
  cpu_baseline  the CPU oracle on a bounded sample of the same pairs
  paths         blocks/s and ms per step of each path
  screening     skipped pairs and missed mass of the value path
  ablation      the 5000-atom screening workload (Coulomb and erfc, values):
                no screening vs analytic bound vs bound + trained network
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_persist_five_ops500_traffic.txt")


def kernel_source_hash() -> str:
    """sha256 of the sources of the persistent kernel (its translation unit and
    the local headers it includes); a stored counter summary is only used for
    the kernel it was taken on"""
    import hashlib
    from paper_1701_06588_amd import build
    tu = os.path.join(ROOT, "paper_1701_06588_amd", "csrc", "shg_persist_d1.hip")
    h = hashlib.sha256()
    for f in sorted(build._deps(tu)):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when there is none or the kernel sources changed since it was taken"""
    if kernel != "shg::k_persist<true>" or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.startswith("    ") and not line.strip().startswith("SQ_"):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash() or "traffic_bytes_per_launch" not in kv:
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(eng, fn, steps, warmup):
    """average ms per call of fn over `steps` calls, HIP events on the library stream"""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(eng.stream)
    wall0 = time.perf_counter()
    for _ in range(steps):
        fn()
    t1.record(eng.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return t0.elapsed_time(t1) / steps, wall


def roofline_of(kernel, ms, nbytes, flops, launches):
    """roofline entry for `launches` launches of one kernel taking `ms` on average"""
    b = nbytes / launches
    f = flops / launches
    t_hbm = b / (HBM_PEAK_GBS * 1e9)
    t_alu = f / (FP64_PEAK_TFLOPS * 1e12)
    s = ms / 1e3
    gbs = b / s / 1e9
    tfl = f / s / 1e12
    if t_alu > t_hbm:
        r = {"bound": "alu", "achieved": round(tfl, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": round(tfl / FP64_PEAK_TFLOPS, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4)}
    r.update({"traffic": None, "kernel": kernel, "avg_launch_ms": round(ms, 4),
              "alg_bytes_per_launch": int(b), "alg_flops_per_launch": int(f),
              "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
              "fp64_tflops": round(tfl, 3), "fp64_frac": round(tfl / FP64_PEAK_TFLOPS, 4),
              "roof_frac": round(max(t_hbm, t_alu) / s, 4)})
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=300000,
                    help="pairs per operator timed on the CPU oracle (0 = skip)")
    ap.add_argument("--no-tune", action="store_true", help="skip loading the tuned tile shapes")
    ap.add_argument("--no-ablation", action="store_true", help="skip the screening ablation")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the three-index overlap and uneven-molecules measurements")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of MIB MiB first (calibrates HBM byte counters)")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the copy / FP64 ceiling measurement")
    ap.add_argument("--paths", default="plain,batched,screened,swap",
                    help="comma list of paths to run (the value needs 'screened')")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this engine runs on one GPU; sharding the pair list over several GPUs is "
                                   "designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1701_06588_amd import inputs, shg, workmodel

    paths = set(args.paths.split(","))
    if args.copy_check > 0:
        src = torch.ones(args.copy_check << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.five_ops500()
    eng = shg.Engine()
    if not args.no_tune:
        from paper_1701_06588_amd import tune
        tune.apply_cache(eng)
    dev = torch.device("cuda")
    dsh = eng.shells(w.shells)
    off, tot = w.out_offsets()
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    out_off = torch.as_tensor(off, device=dev)
    ops = list(inputs.FIVE_OPS)
    n = len(w.pairs)
    blocks_per_step = n * len(ops)
    outs = {op: torch.empty(tot, dtype=torch.float64, device=dev) for op in ops}
    douts = {op: torch.empty(3 * tot, dtype=torch.float64, device=dev) for op in ops}
    res_paths = {}

    # ---- plain per-class launches ----
    def step_plain():
        for op in ops:
            eng.pairs(dsh, op, w.omega[op], pairs, out_off, outs[op], douts[op])

    log("plain path")
    ms_plain, wall_plain = timed(eng, step_plain, args.steps, args.warmup)
    res_paths["plain"] = {"blocks_per_s": round(blocks_per_step / (ms_plain / 1e3), 1), "ms_per_step": round(ms_plain, 4)}

    # ---- batched: one plan per operator (writes the same outputs as plain) ----
    if "batched" in paths:
        log("batched path")
        bplans = [shg.Plan(eng, dsh, op, w.omega[op], pairs, out_off, outs[op], douts[op]) for op in ops]
        modes = []
        for p in bplans:
            p.autotune(3)
            modes.append(p.mode)
        ms_b, _ = timed(eng, lambda: [p.execute() for p in bplans], args.steps, args.warmup)
        res_paths["batched"] = {"blocks_per_s": round(blocks_per_step / (ms_b / 1e3), 1), "ms_per_step": round(ms_b, 4),
                                "modes": dict(zip(ops, modes))}
        for p in bplans:
            p.close()
        # the five operators in one multi-operator plan (one kernel per step)
        mouts = [torch.empty(tot, dtype=torch.float64, device=dev) for _ in ops]
        mdouts = [torch.empty(3 * tot, dtype=torch.float64, device=dev) for _ in ops]
        mplan = shg.MultiPlan(eng, dsh, ops, [w.omega[op] for op in ops], pairs, out_off, mouts, mdouts)
        ms_m, _ = timed(eng, mplan.execute, args.steps, args.warmup)
        res_paths["batched multi-operator"] = {"blocks_per_s": round(blocks_per_step / (ms_m / 1e3), 1),
                                               "ms_per_step": round(ms_m, 4)}
        mplan.close()
        del mouts, mdouts
        step_plain()            # plain outputs back in place (identical anyway)
    torch.cuda.synchronize()

    # ---- batched + screened (the value path) ----
    tau = 1e-10 / blocks_per_step
    souts = {op: torch.empty(tot, dtype=torch.float64, device=dev) for op in ops}
    sdouts = {op: torch.empty(3 * tot, dtype=torch.float64, device=dev) for op in ops}
    log("batched+screened path")
    splans = [shg.Plan(eng, dsh, op, w.omega[op], pairs, out_off, souts[op], sdouts[op], tau=tau) for op in ops]
    for p in splans:
        p.autotune(3)
    ms_s, wall_s = timed(eng, lambda: [p.execute() for p in splans], args.steps, args.warmup)
    value = blocks_per_step / (ms_s / 1e3)
    res_paths["batched+screened"] = {"blocks_per_s": round(value, 1), "ms_per_step": round(ms_s, 4),
                                     "modes": {op: p.mode for op, p in zip(ops, splans)},
                                     "tile_orders": {op: p.tile_order for op, p in zip(ops, splans)}}

    # ---- kept blocks bitwise equal to plain; exact missed mass over skipped blocks ----
    screening = {"tau_blk": tau, "rule": "analytic bound over values and d/dR_a < tau_blk", "per_op": {}}
    bad = 0
    worst = 0.0
    m_tot = dm_tot = 0.0
    for op, p in zip(ops, splans):
        for s_, r_ in ((souts[op], outs[op]), (sdouts[op], douts[op])):
            bad += int(((s_ != r_) & (s_ != 0)).sum().item())
            worst = max(worst, float(((s_ - r_).abs() * (s_ != 0)).max().item() / max(r_.abs().max().item(), 1e-300)))
        mv = float(outs[op][souts[op] == 0].abs().sum().item())
        md = float(douts[op][sdouts[op] == 0].abs().sum().item())
        m_tot += mv
        dm_tot += md
        screening["per_op"][op] = {"skipped": int(p.n_skipped), "missed_mass": mv, "missed_mass_deriv": md}
    screening.update({"skipped": int(sum(p.n_skipped for p in splans)), "candidates": blocks_per_step,
                      "missed_mass": m_tot, "missed_mass_deriv": dm_tot, "kept_blocks_bitwise_equal": bad == 0,
                      "kept_max_diff_rel_to_max": worst,
                      "audit": "every skipped block evaluated exactly (plain path), L1 of its elements"})

    # ---- batched + screened + swap symmetry: evaluate a <= b, fill (b, a) by transposition ----
    a_, b_ = w.pairs[:, 0].astype(np.int64), w.pairs[:, 1].astype(np.int64)
    nsh = int(w.shells.n)
    key = a_ * nsh + b_
    kord = np.argsort(key)
    mir = np.nonzero(a_ > b_)[0]
    pos = np.searchsorted(key[kord], b_[mir] * nsh + a_[mir])
    pos = np.minimum(pos, n - 1)
    partner = kord[pos]
    if "swap" in paths and len(mir) and np.all(key[partner] == b_[mir] * nsh + a_[mir]):
        log("batched+screened+swap path")
        ci = np.nonzero(a_ <= b_)[0]
        cpairs = torch.as_tensor(np.ascontiguousarray(w.pairs[ci], np.int32), device=dev)
        coff = torch.as_tensor(off[ci], device=dev)
        sw_p = torch.as_tensor(np.ascontiguousarray(w.pairs[partner], np.int32), device=dev)
        sw_src = torch.as_tensor(off[partner], device=dev)
        sw_dst = torch.as_tensor(off[mir], device=dev)
        xouts = {op: torch.zeros(tot, dtype=torch.float64, device=dev) for op in ops}
        xdouts = {op: torch.zeros(3 * tot, dtype=torch.float64, device=dev) for op in ops}
        xplans = [shg.Plan(eng, dsh, op, w.omega[op], cpairs, coff, xouts[op], xdouts[op], tau=tau) for op in ops]
        for p in xplans:
            p.autotune(3)

        def step_swap():
            for op, p in zip(ops, xplans):
                p.execute()
                eng.pairs_swap(dsh, sw_p, sw_src, sw_dst, xouts[op], xdouts[op])

        step_swap()
        eng._check(eng.lib.shg_pairs_swap_check(eng.ctx))
        ms_x, _ = timed(eng, step_swap, args.steps, args.warmup)
        ms_xp, _ = timed(eng, lambda: [p.execute() for p in xplans], args.steps, args.warmup)
        # audit: every element against the plain path, |x - r| <= 1e-12 |r| + 1e-14 max(1, max|r|)
        # per operator and component; skipped blocks (both orders) as missed mass
        xbad, xworst, xm, xdm = 0, 0.0, 0.0, 0.0
        for op in ops:
            for x_, r_ in ((xouts[op], outs[op]), (xdouts[op], douts[op])):
                kept = x_ != 0
                tol = 1e-12 * r_.abs() + 1e-14 * max(1.0, r_.abs().max().item())
                xbad += int((((x_ - r_).abs() > tol) & kept).sum().item())
                xworst = max(xworst, float(((x_ - r_).abs() * kept).max().item() / max(r_.abs().max().item(), 1e-300)))
            xm += float(outs[op][xouts[op] == 0].abs().sum().item())
            xdm += float(douts[op][xdouts[op] == 0].abs().sum().item())
        res_paths["batched+screened+swap"] = {
            "blocks_per_s": round(blocks_per_step / (ms_x / 1e3), 1), "ms_per_step": round(ms_x, 4),
            "evaluated_pairs": int(len(ci)), "swapped_pairs": int(len(mir)),
            "plans_ms_per_step": round(ms_xp, 4), "swaps_ms_per_step": round(ms_x - ms_xp, 4),
            "kept_within_tol": xbad == 0, "kept_max_diff_rel_to_max": xworst,
            "missed_mass": xm, "missed_mass_deriv": xdm,
            "note": "screened plans over the pairs with a <= b; the (b, a) blocks by shg_pairs_swap "
                    "(transpose; minus the transpose for d/dR); audited element-wise against the plain path"}
        for p in xplans:
            p.close()
        del xouts, xdouts
        torch.cuda.synchronize()

    # ---- measured device ceilings: plain device copy and FP64 FMA chains ----
    ceilings = None
    if not args.no_ceilings and args.copy_check == 0:   # a byte-counter calibration run keeps one copy only
        log("ceilings")
        cb = 1 << 31
        csrc = torch.ones(cb // 8, dtype=torch.float64, device=dev)
        cdst = torch.empty_like(csrc)
        ms_c, _ = timed(eng, lambda: cdst.copy_(csrc), 5, 1)
        del csrc, cdst
        cout = torch.empty(4096 * 256, dtype=torch.float64, device=dev)
        fl = [0.0]

        def fma_run():
            fl[0] = eng.fp64_ceiling(20000, 4096, cout)

        ms_f, _ = timed(eng, fma_run, 3, 1)
        assert bool(torch.isfinite(cout).all().item())
        del cout
        ceilings = {"copy_gbs": round(2 * cb / (ms_c / 1e3) / 1e9, 1),
                    "copy": "torch copy_ of 2 GiB f64 (read + write counted), HIP events",
                    "fp64_tflops": round(fl[0] / (ms_f / 1e3) / 1e12, 2),
                    "fp64": "shg_fp64_ceiling: 4096 x 256 threads x 20000 rounds x 8 independent FMA chains"}
        torch.cuda.synchronize()

    # ---- roofline of the dominant kernel of the value path ----
    per = []
    skip_mask = {}
    for op, p in zip(ops, splans):
        kept, nbytes = p.stats()
        mask = np.ones(n, bool)
        mask[p.skipped()] = False
        skip_mask[op] = mask
        flops = workmodel.workload_flops(w, op, True, mask)
        kms = p.kernel_ms(5)
        name = "shg::k_persist<true>" if p.mode == "persistent" else f"per-class k_tile<la, lb, true> ({op})"
        per.append((name, kms, nbytes, flops, op))
    groups = {}
    for name, kms, nbytes, flops, op in per:
        g = groups.setdefault(name, [0.0, 0, 0, 0, []])
        g[0] += kms
        g[1] += nbytes
        g[2] += flops
        g[3] += 1
        g[4].append(op)
    name, (kms_sum, nbytes, flops, nl, gops) = max(groups.items(), key=lambda kv: kv[1][0])
    roofline = roofline_of(name, kms_sum / nl, nbytes, flops, nl)
    roofline["launches_averaged"] = {"ops": gops, "per_op_ms": {op: round(k, 4) for _, k, _, _, op in per}}
    roofline["step_share"] = round(kms_sum / ms_s, 3)
    roofline["traffic"] = stored_traffic(name)
    if ceilings:
        roofline["measured_ceilings"] = ceilings
        roofline["frac_of_measured_copy"] = round(roofline["achieved"] / ceilings["copy_gbs"], 4)
        roofline["fp64_frac_of_measured"] = round(roofline["fp64_tflops"] / ceilings["fp64_tflops"], 4)

    for p in splans:
        p.close()
    del souts, sdouts
    torch.cuda.synchronize()

    # ---- screening ablation on the 5000-atom workload (Coulomb, erfc; values) ----
    ablation = None
    if not args.no_ablation:
        from paper_1701_06588_amd import screen
        log("ablation")
        w5 = inputs.screen5000()
        n5 = len(w5.pairs)
        off5, tot5 = w5.out_offsets()
        dsh5 = eng.shells(w5.shells)
        pairs5 = torch.as_tensor(np.ascontiguousarray(w5.pairs, np.int32), device=dev)
        oo5 = torch.as_tensor(off5, device=dev)
        ref5 = torch.empty(tot5, dtype=torch.float64, device=dev)
        got5 = torch.empty(tot5, dtype=torch.float64, device=dev)
        mlp = shg.Mlp(eng, 0)
        mlp.load(screen.MODEL)
        ops5 = list(w5.ops)
        ncand = n5 * len(ops5)
        ablation = {"workload": "screen5000: 5000 atoms, 60 bohr cube, basis as the 500-atom workload, "
                                "ordered atom pairs within 12 bohr, values only",
                    "pairs": n5, "candidates": ncand, "variants": {}}
        steps5 = max(3, args.steps // 2)
        for op in ops5:
            ms_pl, _ = timed(eng, lambda: eng.pairs(dsh5, op, w5.omega[op], pairs5, oo5, ref5), steps5, 1)
            ablation["variants"].setdefault("plain", {})[op] = {"ms": round(ms_pl, 4)}
            torch.cuda.synchronize()
            for tname, tau5 in (("tau_total", 1e-10 / ncand), ("tau_block", 1e-10)):
                for vname, model, tt in (("batched", None, None), ("bound", None, tau5),
                                         ("bound+mlp", mlp, tau5)):
                    if vname == "batched" and tname == "tau_block":
                        continue
                    key = vname if vname == "batched" else f"{vname}@{tname}"
                    log(f"ablation {op} {key}")
                    p = shg.Plan(eng, dsh5, op, w5.omega[op], pairs5, oo5, got5, None, tau=tt, mlp=model)
                    p.autotune(2)
                    ms_v, _ = timed(eng, p.execute, steps5, 1)
                    entry = {"ms": round(ms_v, 4), "skipped": int(p.n_skipped)}
                    if tt is not None:
                        entry["missed_mass"] = float(ref5[got5 == 0].abs().sum().item())
                        entry["kept_bitwise_equal"] = bool(((got5 != ref5) & (got5 != 0)).sum().item() == 0)
                    ablation["variants"].setdefault(key, {})[op] = entry
                    p.close()
        for key, d in ablation["variants"].items():
            ms_sum = sum(v["ms"] for v in d.values())
            d["blocks_per_s"] = round(ncand / (ms_sum / 1e3), 1)
            if all("missed_mass" in v for k, v in d.items() if k in ops5):
                d["missed_mass_total"] = sum(d[o]["missed_mass"] for o in ops5)
        ablation["tau_total"] = 1e-10 / ncand
        mlp.close()
        del ref5, got5
        torch.cuda.synchronize()

    # ---- three-index overlap and uneven molecules (shares of the larger workloads) ----
    extra = None
    if not args.no_extra:
        extra = {}
        log("three-index overlap")
        n3 = 250
        w3 = inputs.aab2000(n_atoms=n3, box=40.0 * (n3 / 2000) ** (1 / 3))
        off3, tot3 = w3.out_offsets()
        orb3, aux3 = eng.shells(w3.shells), eng.shells(w3.aux)
        tri3 = torch.as_tensor(np.ascontiguousarray(w3.triples, np.int32), device=dev)
        oo3 = torch.as_tensor(off3, device=dev)
        o3 = torch.empty(tot3, dtype=torch.float64, device=dev)
        d3 = torch.empty(3 * tot3, dtype=torch.float64, device=dev)
        nt3 = len(w3.triples)
        sz = w3.shells.l
        b3 = int(workmodel.triple_bytes(sz[w3.triples[:, 0]], w3.aux.l[w3.triples[:, 1]],
                                        sz[w3.triples[:, 2]], True).sum())
        steps3 = max(2, args.steps // 3)
        ms3, _ = timed(eng, lambda: eng.aab(orb3, aux3, tri3, oo3, o3, d3), steps3, 1)
        extra["aab"] = {"workload": f"aab2000 share: {n3} atoms at the 2000-atom density (40 bohr cube), orbital "
                                    "l 0..3 K 5, RI l 0..6 uncontracted, triples (orbital on X, RI on X, orbital "
                                    "on Y) of atom pairs within 10 bohr, values + d/dR_A",
                        "triples": nt3, "ms_per_call": round(ms3, 4),
                        "triples_per_s": round(nt3 / (ms3 / 1e3), 1),
                        "alg_bytes_per_call": b3, "hbm_gbs": round(b3 / (ms3 / 1e3) / 1e9, 1),
                        "hbm_frac": round(b3 / (ms3 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del o3, d3
        torch.cuda.synchronize()
        log("r_a^2n two-center integrals")
        b_r2n = int(workmodel.workload_bytes(w, True))
        r2n = {"workload": "five_ops500 pair list (all shell pairs of the 500-atom workload), values + d/dR_a",
               "pairs": n, "alg_bytes_per_call": b_r2n}
        steps5 = max(2, args.steps // 3)
        for nr in (1, 3, 5):
            ms5, _ = timed(eng, lambda: eng.pairs_r2n(dsh, nr, pairs, out_off, outs[ops[0]], douts[ops[0]]),
                           steps5, 1)
            r2n[f"n{nr}"] = {"ms_per_call": round(ms5, 4), "blocks_per_s": round(n / (ms5 / 1e3), 1),
                             "hbm_frac": round(b_r2n / (ms5 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        rplan = shg.Plan(eng, dsh, "r2n", 0.0, pairs, out_off, outs[ops[0]], douts[ops[0]], nr=3)
        rplan.autotune(2)
        ms8, _ = timed(eng, rplan.execute, steps5, 1)
        r2n["n3_batched"] = {"ms_per_call": round(ms8, 4), "blocks_per_s": round(n / (ms8 / 1e3), 1),
                             "mode": rplan.mode}
        rplan.close()
        extra["r2n"] = r2n
        ms6, _ = timed(eng, lambda: eng.pairs(dsh, "gcoulomb", 0.7, pairs, out_off, outs[ops[0]], douts[ops[0]]),
                       steps5, 1)
        gplan = shg.Plan(eng, dsh, "gcoulomb", 0.7, pairs, out_off, outs[ops[0]], douts[ops[0]])
        gplan.autotune(2)
        ms7, _ = timed(eng, gplan.execute, steps5, 1)
        gmode = gplan.mode
        gplan.close()
        extra["gcoulomb"] = {"workload": "five_ops500 pair list, exp(-0.7 r^2)/r, values + d/dR_a, shg_pairs_deriv",
                             "pairs": n, "ms_per_call": round(ms6, 4), "blocks_per_s": round(n / (ms6 / 1e3), 1),
                             "hbm_frac": round(b_r2n / (ms6 / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                             "batched": {"ms_per_call": round(ms7, 4), "blocks_per_s": round(n / (ms7 / 1e3), 1),
                                         "mode": gmode}}
        torch.cuda.synchronize()
        log("uneven molecules")
        w4 = inputs.molecules256(n_mol=32)
        off4, tot4 = w4.out_offsets()
        dsh4 = eng.shells(w4.shells)
        p4 = torch.as_tensor(np.ascontiguousarray(w4.pairs, np.int32), device=dev)
        oo4 = torch.as_tensor(off4, device=dev)
        o4 = torch.empty(tot4, dtype=torch.float64, device=dev)
        d4 = torch.empty(3 * tot4, dtype=torch.float64, device=dev)
        n4 = len(w4.pairs)
        m4 = {"plain": 0.0, "batched": 0.0}
        modes4 = {}
        steps4 = max(2, args.steps // 3)
        for op in ops:
            ms_p, _ = timed(eng, lambda: eng.pairs(dsh4, op, w4.omega[op], p4, oo4, o4, d4), steps4, 1)
            pl = shg.Plan(eng, dsh4, op, w4.omega[op], p4, oo4, o4, d4)
            pl.autotune(2)
            modes4[op] = pl.mode
            ms_b, _ = timed(eng, pl.execute, steps4, 1)
            pl.close()
            m4["plain"] += ms_p
            m4["batched"] += ms_b
        extra["molecules"] = {"workload": "molecules256 share: 32 molecules of 10..400 atoms (log-uniform), "
                                          "500-atom-workload basis, unordered intra-molecule shell pairs within "
                                          "12 bohr, 5 operators, values + d/dR_a",
                              "pairs": n4, "blocks_per_step": n4 * len(ops),
                              "plain_blocks_per_s": round(n4 * len(ops) / (m4["plain"] / 1e3), 1),
                              "batched_blocks_per_s": round(n4 * len(ops) / (m4["batched"] / 1e3), 1),
                              "speedup": round(m4["plain"] / m4["batched"], 3), "modes": modes4}
        del o4, d4
        torch.cuda.synchronize()

    # ---- CPU oracle on a bounded sample of the same pairs ----
    cpu = None
    if args.cpu_sample > 0:
        import oracle
        log("cpu baseline")
        rng = np.random.default_rng(0)
        idx = np.sort(rng.choice(n, min(args.cpu_sample, n), replace=False))
        c0 = time.perf_counter()
        for op in ops:
            oracle.pairs(w.shells, op, w.omega[op], w.pairs[idx], deriv=True)
        cdt = time.perf_counter() - c0
        cpu = {"value": round(len(idx) * len(ops) / cdt, 1), "unit": "blocks/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{len(idx)} random shell pairs of the same workload x 5 operators, values + d/dR_a, "
                         f"double-precision Obara-Saika oracle, {cdt:.1f} s"}

    res = {
        "metric": "contracted shell-pair blocks/sec (FP64, <=1e-12 rel err), batched+screened vs plain",
        "value": round(value, 1),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_s, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "five_ops500: 500 atoms, 20 bohr cube, 4 shells/atom l 0..4 K 1..7, "
                               "ordered atom pairs within 12 bohr",
                   "pairs": n, "operators": ops, "derivatives": True, "path": "batched+screened",
                   "blocks_per_step": blocks_per_step},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": {
            "what": "the paper's OS/SHG speed-up ratios (Table 3, MOLOPT basis sets, integrals + derivatives), "
                    "measured in CP2K on one Xeon E5-2697v3 (Haswell); context only, other hardware and code",
            "os_over_shg_int_dev_range": {"overlap": [2.4, 10.3], "coulomb": [6.2, 31.6], "erf": [6.0, 31.7],
                                          "erfc": [5.4, 29.5], "gauss": [6.7, 32.5], "aab": [7.2, 10.5],
                                          "gcoulomb": [5.0, 25.4], "r2n_n1": [2.7, 18.6], "r2n_n5": [10.5, 79.9]},
            "gpu_shg_over_cpu_oracle": (round(value / cpu["value"], 1) if cpu and cpu.get("value") else None)},
        "paths": res_paths,
        "speedup_vs_plain": round(ms_plain / ms_s, 3),
        "screening": screening,
        "ablation": ablation,
        "extra": extra,
        "wall_s_timed": round(wall_s, 3),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
