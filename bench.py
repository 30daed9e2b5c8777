"""Benchmark: contracted shell-pair blocks per second on one MI355X.

Workload (one "step"): the uneven-molecules serving workload at full size --
256 molecules of 10..400 atoms (log-uniform), 4 shells per atom (l 0..4,
K 1..7, exponents log-uniform [0.05, 50]), every unordered intra-molecule shell
pair within 12 bohr (30.9e6 shell pairs), evaluated for all five operators
(overlap, Coulomb, erfc(0.11 r)/r, erf(0.33 r)/r, exp(-r^2)) with values and
d/dR_a. Inputs are synthetic (seeded) and resident in HBM before the timed
region; the five operators' outputs (124 GB) stay resident.

Paths over the same pair list, each timed with HIP events on the library
stream over --steps steps after --warmup untimed ones:
  plain             shg_pairs_deriv per operator (binning + one launch per class)
  batched           one recorded plan per operator (binned once, hipGraph
                    replay of the persistent class-binned kernel)
  batched+screened  the value path: screened plans, which decide on every
                    execution, on the device, which pairs to evaluate (pairs
                    whose analytic bound over values and d/dR_a is below
                    tau_blk = 1e-10 / N_candidates are skipped and their blocks
                    zeroed); the screening stage is inside the timed region
`value` is the batched+screened rate in candidate blocks per second (every
block of the step counts, skipped or not). Kept blocks are checked bitwise
against the plain path; the missed mass is exact (L1 of the plain path's values
and derivatives over every skipped block).

Prints ONE JSON line. Fields beyond the common contract:
  roofline      k_persist<true> of the value path: its duration measured live in
                the timed replays (HIP events on the library stream around each
                plan's evaluation graph), algorithmic bytes (and flops) per
                launch from the kept pairs of each plan
  cpu_baseline  the CPU oracle on a bounded sample of the same pairs (all host
                threads, and one thread on a smaller sample)
  paths         blocks/s and ms per step of each path
  screening     skipped pairs and missed mass of the value path
  extra         the other workloads: 200 isolated overlap pairs (launch
                latency), the 500-atom five-operator workload, the three-index
                overlap of the 2000-atom RI workload at full size, the
                5000-atom screening workload with the trained network, and the
                next-row operators
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_persist_molecules256_traffic.txt")


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


def stored_traffic(args):
    """HBM bytes per evaluation (the heavy- and light-class launches of k_persist<true>)
    on this workload from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on a plain copy), or None when there is none, the
    kernel sources changed since, or the run is not the one the counters were
    taken on (the full 256 molecules, round-robin tile order)"""
    if args.n_mol != 256 or args.tile_order != "round-robin" or not os.path.exists(TRAFFIC_FILE):
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


def oracle_rate(fn, units, unit, sample, reps=1):
    """the CPU oracle's rate on a bounded sample: fn() evaluates `units` blocks
    (or triples) on all host threads; reps calls are timed together"""
    import oracle
    c0 = time.perf_counter()
    for _ in range(reps):
        fn()
    dt = time.perf_counter() - c0
    return {"value": round(units * reps / dt, 1), "unit": unit, "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{sample}, {dt:.2f} s"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def upload(eng, w):
    import numpy as np
    import torch
    dev = torch.device("cuda")
    off, tot = w.out_offsets()
    return (eng.shells(w.shells), torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev),
            torch.as_tensor(off, device=dev), off, tot)


def make_plans(shg, eng, dsh, ops, omega, pairs, out_off, outs, douts, tile_order, tau=None, mlp=None):
    plans = []
    for op in ops:
        p = shg.Plan(eng, dsh, op, omega[op], pairs, out_off, outs[op], douts[op] if douts else None,
                     shg.PLAN_PERSISTENT, tau=tau, mlp=mlp)
        if tile_order == "auto":
            p.autotune(3)
        else:
            p.set_tile_order(tile_order)
        plans.append(p)
    return plans


def compare_chunked(got, ref, chunk=1 << 27):
    """(elements of got that are neither zero nor equal to ref, L1 of ref where got is zero),
    over slices so that no temporary exceeds `chunk` elements"""
    bad, mass = 0, 0.0
    for i in range(0, got.numel(), chunk):
        g, r = got[i:i + chunk], ref[i:i + chunk]
        z = g == 0
        bad += int(((g != r) & ~z).sum().item())
        mass += float((r.abs() * z).sum().item())
    return bad, mass


def audit(outs, refs_fn, ops, douts=None):
    """kept blocks bitwise equal to the plain path, exact missed mass over the zeroed elements"""
    import torch
    res = {"per_op": {}, "kept_bitwise_equal": True, "missed_mass": 0.0, "missed_mass_deriv": 0.0}
    for op in ops:
        ref, dref = refs_fn(op)
        torch.cuda.synchronize()
        bad, mv = compare_chunked(outs[op], ref)
        md = 0.0
        if douts is not None:
            b2, md = compare_chunked(douts[op], dref)
            bad += b2
        res["per_op"][op] = {"missed_mass": mv, "missed_mass_deriv": md, "mismatched_kept_elements": bad}
        res["kept_bitwise_equal"] &= bad == 0
        res["missed_mass"] += mv
        res["missed_mass_deriv"] += md
        del ref, dref
        torch.cuda.synchronize()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=20000,
                    help="pairs timed on the CPU oracle with all host threads (x 5 operators; 0 = skip)")
    ap.add_argument("--cpu-sample-1core", type=int, default=2000,
                    help="pairs timed on the CPU oracle with one thread (x 5 operators; 0 = skip)")
    ap.add_argument("--tile-order", default="round-robin",
                    choices=["round-robin", "alternating", "heaviest-first", "auto"],
                    help="tile order of the plans' persistent queue (auto: timed by the plan autotuner)")
    ap.add_argument("--no-extra", action="store_true", help="skip the measurements of the other workloads")
    ap.add_argument("--extras", default="all",
                    help="comma list of the other workloads to measure: overlap200, five_ops500, aab2000, "
                         "molopt_sets, screen5000 (default all)")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of MIB MiB first (calibrates HBM byte counters)")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the copy / FP64 ceiling measurement")
    ap.add_argument("--paths", default="plain,batched,screened",
                    help="comma list of paths to run (the value needs 'screened')")
    ap.add_argument("--n-mol", type=int, default=256, help="molecules of the workload (256 = full size)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this engine runs on one GPU; sharding the pair list over several GPUs is "
                                   "designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1701_06588_amd import inputs, shg, tune, workmodel

    paths = set(args.paths.split(","))
    if args.copy_check > 0:
        src = torch.ones(args.copy_check << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log("workload molecules256")
    w = inputs.molecules256(n_mol=args.n_mol)
    eng = shg.Engine()
    tune.apply_cache(eng)
    dev = torch.device("cuda")
    dsh, pairs, out_off, off, tot = upload(eng, w)
    ops = list(inputs.FIVE_OPS)
    n = len(w.pairs)
    blocks_per_step = n * len(ops)
    outs = {op: torch.empty(tot, dtype=torch.float64, device=dev) for op in ops}
    douts = {op: torch.empty(3 * tot, dtype=torch.float64, device=dev) for op in ops}
    res_paths = {}

    # ---- plain per-class launches ----
    ms_plain = None
    if "plain" in paths:
        def step_plain():
            for op in ops:
                eng.pairs(dsh, op, w.omega[op], pairs, out_off, outs[op], douts[op])

        log("plain path")
        ms_plain, _ = timed(eng, step_plain, args.steps, args.warmup)
        res_paths["plain"] = {"blocks_per_s": round(blocks_per_step / (ms_plain / 1e3), 1),
                              "ms_per_step": round(ms_plain, 4)}

    # ---- batched: one plan per operator (writes the same outputs as plain) ----
    if "batched" in paths:
        log("batched path")
        bplans = make_plans(shg, eng, dsh, ops, w.omega, pairs, out_off, outs, douts, args.tile_order)
        ms_b, _ = timed(eng, lambda: [p.execute() for p in bplans], args.steps, args.warmup)
        res_paths["batched"] = {"blocks_per_s": round(blocks_per_step / (ms_b / 1e3), 1),
                                "ms_per_step": round(ms_b, 4), "tile_orders": [p.tile_order for p in bplans]}
        for p in bplans:
            p.close()
        torch.cuda.synchronize()

    # ---- batched + screened (the value path), kernel time measured in the timed replays ----
    tau = 1e-10 / blocks_per_step
    log("batched+screened path")
    splans = make_plans(shg, eng, dsh, ops, w.omega, pairs, out_off, outs, douts, args.tile_order, tau=tau)
    for p in splans:
        p.execute()
    torch.cuda.synchronize()
    for p in splans:
        p.time_kernels(True)
    ms_s, wall_s = timed(eng, lambda: [p.execute() for p in splans], args.steps, args.warmup)
    value = blocks_per_step / (ms_s / 1e3)
    kern = []
    for op, p in zip(ops, splans):
        kms, cnt = p.kernel_time()
        p.time_kernels(False)
        kept, nbytes = p.stats()
        kern.append((op, kms / max(cnt, 1), cnt, kept, nbytes))
    res_paths["batched+screened"] = {"blocks_per_s": round(value, 1), "ms_per_step": round(ms_s, 4),
                                     "tile_orders": [p.tile_order for p in splans]}
    skip_ids = {op: p.skipped() for op, p in zip(ops, splans)}
    skipped = {op: int(ids.size) for op, ids in skip_ids.items()}
    for p in splans:
        p.close()
    torch.cuda.synchronize()

    # ---- audit against the plain path, one operator at a time ----
    log("audit")

    def plain_ref(op):
        r = torch.empty(tot, dtype=torch.float64, device=dev)
        d = torch.empty(3 * tot, dtype=torch.float64, device=dev)
        eng.pairs(dsh, op, w.omega[op], pairs, out_off, r, d)
        return r, d

    screening = audit(outs, plain_ref, ops, douts)
    for op in ops:
        screening["per_op"][op]["skipped"] = skipped[op]
    screening.update({"tau_blk": tau, "rule": "analytic bound over values and d/dR_a < tau_blk, decided on "
                                              "the device in every replay",
                      "skipped": int(sum(skipped.values())), "candidates": blocks_per_step,
                      "audit": "every skipped block evaluated exactly (plain path), L1 of its elements"})

    # ---- roofline of the dominant kernel: k_persist<true>, one launch per operator ----
    nb_sum = sum(k[4] for k in kern)
    ms_sum = sum(k[1] for k in kern)
    fl_sum = 0
    for op in ops:
        mask = np.ones(n, bool)
        mask[skip_ids[op]] = False
        fl_sum += workmodel.workload_flops(w, op, True, mask)
    b_launch = nb_sum / len(ops)
    f_launch = fl_sum / len(ops)
    ms_launch = ms_sum / len(ops)
    gbs = b_launch / (ms_launch / 1e3) / 1e9
    tfl = f_launch / (ms_launch / 1e3) / 1e12
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": stored_traffic(args),
                "kernel": "shg::k_persist<true, heavy> + shg::k_persist<true, light> (one evaluation: the "
                          "heavy-class and the light-class persistent launches of a plan)",
                "avg_launch_ms": round(ms_launch, 4),
                "alg_bytes_per_launch": int(b_launch), "alg_flops_per_launch": int(f_launch),
                "fp64_tflops": round(tfl, 3), "fp64_frac": round(tfl / FP64_PEAK_TFLOPS, 4),
                "per_op_ms": {k[0]: round(k[1], 4) for k in kern},
                "timed_launches": {k[0]: k[2] for k in kern},
                "step_share": round(ms_sum / ms_s, 4),
                "how": "HIP events on the library stream around each screened plan's evaluation graph in every "
                       "timed replay; bytes = 8 (2la+1)(2lb+1) x 4 + 16 per kept pair (workmodel)"}
    if b_launch / (HBM_PEAK_GBS * 1e9) < f_launch / (FP64_PEAK_TFLOPS * 1e12):
        roofline.update({"bound": "alu", "achieved": round(tfl, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tfl / FP64_PEAK_TFLOPS, 4)})
    roofline["step_frac_hbm"] = round(sum(k[4] for k in kern) / (ms_s / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    del outs, douts
    torch.cuda.empty_cache()

    # ---- measured device ceilings: plain device copy and FP64 FMA chains ----
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
        del cout
        ceil = {"copy_gbs": round(2 * cb / (ms_c / 1e3) / 1e9, 1),
                "copy": "torch copy_ of 2 GiB f64 (read + write counted), HIP events",
                "fp64_tflops": round(fl[0] / (ms_f / 1e3) / 1e12, 2),
                "fp64": "shg_fp64_ceiling: 4096 x 256 threads x 20000 rounds x 8 independent FMA chains"}
        roofline["measured_ceilings"] = ceil
        roofline["frac_of_measured_copy"] = round(gbs / ceil["copy_gbs"], 4)
        roofline["fp64_frac_of_measured"] = round(tfl / ceil["fp64_tflops"], 4)
        torch.cuda.synchronize()

    extra = None if args.no_extra else run_extras(args, eng, shg, inputs, workmodel, np, torch)

    # ---- CPU oracle on bounded samples of the same pairs ----
    cpu = None
    if args.cpu_sample > 0:
        import oracle
        log("cpu baseline")
        rng = np.random.default_rng(0)
        idx = np.sort(rng.choice(n, min(args.cpu_sample, n), replace=False))
        nthr = oracle.num_threads()
        c0 = time.perf_counter()
        for op in ops:
            oracle.pairs(w.shells, op, w.omega[op], w.pairs[idx], deriv=True)
        cdt = time.perf_counter() - c0
        cpu = {"value": round(len(idx) * len(ops) / cdt, 1), "unit": "blocks/s", "cores": nthr, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{len(idx)} random shell pairs of the same workload x 5 operators, values + d/dR_a, "
                         f"double-precision Obara-Saika oracle on {nthr} threads, {cdt:.1f} s"}
        if args.cpu_sample_1core > 0:
            idx1 = idx[:args.cpu_sample_1core]
            oracle.set_num_threads(1)
            c0 = time.perf_counter()
            for op in ops:
                oracle.pairs(w.shells, op, w.omega[op], w.pairs[idx1], deriv=True)
            c1 = time.perf_counter() - c0
            oracle.set_num_threads(nthr)
            cpu["one_core"] = {"value": round(len(idx1) * len(ops) / c1, 1), "unit": "blocks/s", "cores": 1,
                               "sample": f"the first {len(idx1)} pairs of that sample x 5 operators, {c1:.1f} s"}

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
        "config": {"workload": f"molecules256: {args.n_mol} uneven molecules of 10..400 atoms (log-uniform), "
                               "4 shells/atom l 0..4 K 1..7, unordered intra-molecule shell pairs within 12 bohr"
                               + (" (full size)" if args.n_mol == 256 else " (share)"),
                   "pairs": n, "atoms": int(w.n_atoms), "operators": ops, "derivatives": True,
                   "path": "batched+screened", "blocks_per_step": blocks_per_step,
                   "tile_order": args.tile_order},
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
        "speedup_vs_plain": round(ms_plain / ms_s, 3) if ms_plain else None,
        "screening": screening,
        "extra": extra,
        "wall_s_timed": round(wall_s, 3),
    }
    print(json.dumps(res), flush=True)


def family_set_extra(eng, shg, inputs, np, torch, natoms, density, kinds, cutoff, steps):
    """Coulomb integrals + d/dR_A of MOLOPT family sets (Tables S2-S5) for atoms at
    `density` (per bohr^3) in a cube, all ordered atom pairs within `cutoff`:
    shg_set_pairs against shg_pairs_deriv on every function pair of the same set
    pairs (the functions taken as shells)"""
    from paper_1701_06588_amd import basis_molopt as bm
    dev = torch.device("cuda")
    rng = np.random.default_rng(1006)
    side = (natoms / density) ** (1.0 / 3.0)
    pos = rng.uniform(0.0, side, size=(natoms, 3))
    names = [kinds[i % len(kinds)] for i in range(natoms)]
    st = bm.make_sets(pos, names)
    sp = np.ascontiguousarray(inputs.atom_pairs_within(pos, cutoff), np.int32)
    nsgf = st.nsgf()
    sz = nsgf[sp[:, 0]] * nsgf[sp[:, 1]]
    off = np.zeros(len(sz), np.int64)
    off[1:] = np.cumsum(sz[:-1])
    tot = int(sz.sum())
    ds = eng.sets(st)
    tsp = torch.as_tensor(sp, device=dev)
    too = torch.as_tensor(off, device=dev)
    out = torch.empty(tot, dtype=torch.float64, device=dev)
    dout = torch.empty(3 * tot, dtype=torch.float64, device=dev)
    ms_set, _ = timed(eng, lambda: eng.set_pairs(ds, "coulomb", 0.0, tsp, too, out, dout), steps, 1)
    # the same function pairs through the shell path
    sh, first = st.as_shells()
    na = st.nfun[sp[:, 0]].astype(np.int64)
    nb = st.nfun[sp[:, 1]].astype(np.int64)
    cnt = na * nb
    rep = np.repeat(np.arange(len(sp)), cnt)
    local = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    fa = first[sp[rep, 0]] + local // nb[rep]
    fb = first[sp[rep, 1]] + local % nb[rep]
    fp = np.ascontiguousarray(np.stack([fa, fb], axis=1), np.int32)
    fsz = (2 * sh.l[fp[:, 0]].astype(np.int64) + 1) * (2 * sh.l[fp[:, 1]].astype(np.int64) + 1)
    foff = np.zeros(len(fsz), np.int64)
    foff[1:] = np.cumsum(fsz[:-1])
    assert int(fsz.sum()) == tot
    dsh = eng.shells(sh)
    tfp = torch.as_tensor(fp, device=dev)
    tfo = torch.as_tensor(foff, device=dev)
    ms_sh, _ = timed(eng, lambda: eng.pairs(dsh, "coulomb", 0.0, tfp, tfo, out, dout), steps, 1)
    nbytes = 4 * tot * 8 + 16 * len(sp)
    del out, dout
    torch.cuda.empty_cache()
    return {"workload": f"{natoms} atoms ({'/'.join(kinds)}) at {density} bohr^-3, ordered atom pairs within "
                        f"{cutoff} bohr, Coulomb values + d/dR_A",
            "set_pairs": len(sp), "function_pairs": len(fp), "elements": tot,
            "set_path_ms": round(ms_set, 4), "shell_path_ms": round(ms_sh, 4),
            "speedup_set_over_shells": round(ms_sh / ms_set, 3),
            "function_pair_blocks_per_s": round(len(fp) / (ms_set / 1e3), 1),
            "hbm_frac": round(nbytes / (ms_set / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_extras(args, eng, shg, inputs, workmodel, np, torch):
    dev = torch.device("cuda")
    extra = {}
    steps = max(3, args.steps // 2)
    sel = None if args.extras == "all" else set(args.extras.split(","))

    def want(name):
        return sel is None or name in sel

    # ---- 200 isolated overlap pairs: launch latency, single call vs graph replay ----
    if want("overlap200"):
        log("extra: overlap200 latency")
        w1 = inputs.overlap200()
        dsh1, p1, oo1, _, tot1 = upload(eng, w1)
        o1 = torch.empty(tot1, dtype=torch.float64, device=dev)
        ms_single, _ = timed(eng, lambda: eng.pairs(dsh1, "overlap", 0.0, p1, oo1, o1), 50, 5)
        pl1 = shg.Plan(eng, dsh1, "overlap", 0.0, p1, oo1, o1, None, shg.PLAN_PERSISTENT)
        ms_graph, _ = timed(eng, pl1.execute, 200, 10)
        pl1.close()
        extra["overlap200"] = {"workload": "200 isolated atom pairs, one shell per center, l 0..2, K 3, overlap values",
                               "blocks": len(w1.pairs),
                               "single_call_us": round(ms_single * 1e3, 2),
                               "single_call_blocks_per_s": round(len(w1.pairs) / (ms_single / 1e3), 1),
                               "graph_replay_us": round(ms_graph * 1e3, 2),
                               "graph_replay_blocks_per_s": round(len(w1.pairs) / (ms_graph / 1e3), 1),
                               "note": "latency bound: shg_pairs bins and synchronises once per call; a plan replays "
                                       "its graphs with no host synchronisation"}
        if args.cpu_sample > 0:
            import oracle
            extra["overlap200"]["cpu_oracle"] = oracle_rate(
                lambda: oracle.pairs(w1.shells, "overlap", 0.0, w1.pairs), len(w1.pairs), "blocks/s",
                "all 200 pairs, overlap values, 50 repetitions", reps=50)

    # ---- the 500-atom five-operator workload ----
    if want("five_ops500"):
        log("extra: five_ops500")
        w2 = inputs.five_ops500()
        dsh2, p2, oo2, off2, tot2 = upload(eng, w2)
        ops = list(inputs.FIVE_OPS)
        n2 = len(w2.pairs)
        o2 = {op: torch.empty(tot2, dtype=torch.float64, device=dev) for op in ops}
        d2 = {op: torch.empty(3 * tot2, dtype=torch.float64, device=dev) for op in ops}
        ms_p2, _ = timed(eng, lambda: [eng.pairs(dsh2, op, w2.omega[op], p2, oo2, o2[op], d2[op]) for op in ops],
                         steps, 2)
        tau2 = 1e-10 / (n2 * 5)
        sp2 = make_plans(shg, eng, dsh2, ops, w2.omega, p2, oo2, o2, d2, args.tile_order, tau=tau2)
        ms_s2, _ = timed(eng, lambda: [p.execute() for p in sp2], steps, 2)
        for p in sp2:
            p.close()
        extra["five_ops500"] = {"workload": "500 atoms, 20 bohr cube, 4 shells/atom l 0..4 K 1..7, ordered atom pairs "
                                            "within 12 bohr, 5 operators, values + d/dR_a",
                                "pairs": n2, "blocks_per_step": n2 * 5,
                                "plain_blocks_per_s": round(n2 * 5 / (ms_p2 / 1e3), 1),
                                "batched_screened_blocks_per_s": round(n2 * 5 / (ms_s2 / 1e3), 1),
                                "speedup": round(ms_p2 / ms_s2, 3)}
        if args.cpu_sample > 0:
            import oracle
            i2 = np.sort(np.random.default_rng(0).choice(n2, min(20000, n2), replace=False))
            extra["five_ops500"]["cpu_oracle"] = oracle_rate(
                lambda: [oracle.pairs(w2.shells, op, w2.omega[op], w2.pairs[i2], deriv=True) for op in ops],
                len(i2) * len(ops), "blocks/s", f"{len(i2)} random pairs x 5 operators, values + d/dR_a")
        # swap symmetry on this ordered list: screened plans over a <= b, (b, a) by transposition
        a_, b_ = w2.pairs[:, 0].astype(np.int64), w2.pairs[:, 1].astype(np.int64)
        nsh = int(w2.shells.n)
        key = a_ * nsh + b_
        kord = np.argsort(key)
        mir = np.nonzero(a_ > b_)[0]
        pos = np.minimum(np.searchsorted(key[kord], b_[mir] * nsh + a_[mir]), n2 - 1)
        partner = kord[pos]
        if len(mir) and np.all(key[partner] == b_[mir] * nsh + a_[mir]):
            ci = np.nonzero(a_ <= b_)[0]
            cp = torch.as_tensor(np.ascontiguousarray(w2.pairs[ci], np.int32), device=dev)
            coff = torch.as_tensor(off2[ci], device=dev)
            sw_p = torch.as_tensor(np.ascontiguousarray(w2.pairs[partner], np.int32), device=dev)
            sw_src = torch.as_tensor(off2[partner], device=dev)
            sw_dst = torch.as_tensor(off2[mir], device=dev)
            xo = {op: torch.zeros(tot2, dtype=torch.float64, device=dev) for op in ops}
            xd = {op: torch.zeros(3 * tot2, dtype=torch.float64, device=dev) for op in ops}
            xp = make_plans(shg, eng, dsh2, ops, w2.omega, cp, coff, xo, xd, args.tile_order, tau=tau2)

            def step_swap():
                for op, p in zip(ops, xp):
                    p.execute()
                    eng.pairs_swap(dsh2, sw_p, sw_src, sw_dst, xo[op], xd[op])

            step_swap()
            eng._check(eng.lib.shg_pairs_swap_check(eng.ctx))
            ms_x, _ = timed(eng, step_swap, steps, 2)
            xbad = 0
            for op in ops:
                for x_, r_ in ((xo[op], o2[op]), (xd[op], d2[op])):
                    tol = 1e-12 * r_.abs() + 1e-14 * max(1.0, r_.abs().max().item())
                    xbad += int((((x_ - r_).abs() > tol) & (x_ != 0)).sum().item())
            for p in xp:
                p.close()
            extra["five_ops500"]["screened_swap_blocks_per_s"] = round(n2 * 5 / (ms_x / 1e3), 1)
            extra["five_ops500"]["swap_within_tol"] = xbad == 0
            del xo, xd
        # next-row operators on the same pair list
        b_r2n = int(workmodel.workload_bytes(w2, True))
        r2n = {"pairs": n2, "alg_bytes_per_call": b_r2n}
        for nr in (1, 3, 5):
            ms5, _ = timed(eng, lambda: eng.pairs_r2n(dsh2, nr, p2, oo2, o2[ops[0]], d2[ops[0]]), steps, 1)
            r2n[f"n{nr}"] = {"ms_per_call": round(ms5, 4), "blocks_per_s": round(n2 / (ms5 / 1e3), 1),
                             "hbm_frac": round(b_r2n / (ms5 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        extra["r2n_five_ops500"] = r2n
        ms6, _ = timed(eng, lambda: eng.pairs(dsh2, "gcoulomb", 0.7, p2, oo2, o2[ops[0]], d2[ops[0]]), steps, 1)
        extra["gcoulomb_five_ops500"] = {"ms_per_call": round(ms6, 4), "blocks_per_s": round(n2 / (ms6 / 1e3), 1),
                                         "hbm_frac": round(b_r2n / (ms6 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del o2, d2
        torch.cuda.empty_cache()

    # ---- three-index overlap, full 2000-atom RI workload, one call ----
    if want("aab2000"):
        log("extra: aab2000 full size")
        w3 = inputs.aab2000()
        off3, tot3 = w3.out_offsets()
        orb3, aux3 = eng.shells(w3.shells), eng.shells(w3.aux)
        tri3 = torch.as_tensor(np.ascontiguousarray(w3.triples, np.int32), device=dev)
        oo3 = torch.as_tensor(off3, device=dev)
        o3 = torch.empty(tot3, dtype=torch.float64, device=dev)
        d3 = torch.empty(3 * tot3, dtype=torch.float64, device=dev)
        nt3 = len(w3.triples)
        sz = w3.shells.l
        b3 = int(workmodel.triple_bytes(sz[w3.triples[:, 0]], w3.aux.l[w3.triples[:, 1]], sz[w3.triples[:, 2]],
                                        True).sum())
        ms3, _ = timed(eng, lambda: eng.aab(orb3, aux3, tri3, oo3, o3, d3), 3, 1)
        finite = bool(torch.isfinite(o3).all().item()) and bool(torch.isfinite(d3).all().item())
        extra["aab2000"] = {"workload": "2000 atoms, 40 bohr cube, orbital l 0..3 K 5, RI l 0..6 uncontracted, "
                                        "triples (orbital on X, RI on X, orbital on Y) of ordered atom pairs within "
                                        "10 bohr, values + d/dR_A, full size in one shg_aab call",
                            "triples": nt3, "output_gb": round(4 * tot3 * 8 / 1e9, 2), "ms_per_call": round(ms3, 3),
                            "triples_per_s": round(nt3 / (ms3 / 1e3), 1), "alg_bytes_per_call": b3,
                            "hbm_gbs": round(b3 / (ms3 / 1e3) / 1e9, 1),
                            "hbm_frac": round(b3 / (ms3 / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "all_finite": finite}
        if args.cpu_sample > 0:
            import oracle
            i3 = np.sort(np.random.default_rng(0).choice(nt3, min(5000, nt3), replace=False))
            extra["aab2000"]["cpu_oracle"] = oracle_rate(
                lambda: oracle.aab(w3.shells, w3.aux, w3.triples[i3], deriv=True), len(i3), "triples/s",
                f"{len(i3)} random triples, values + d/dR_A")
        del o3, d3, tri3, oo3
        torch.cuda.empty_cache()

    # ---- family sets on the paper's MOLOPT data: set path vs the same functions as shells ----
    if want("molopt_sets"):
        log("extra: MOLOPT family sets")
        extra["molopt_sets"] = {}
        for name, natoms, dens, kinds, cut in (("water", 12000, 0.0148, ("O-DZVP", "H-DZVP", "H-DZVP"), 10.0),
                                               ("copper", 4000, 0.0126, ("Cu-DZVP",), 9.0)):
            extra["molopt_sets"][name] = family_set_extra(eng, shg, inputs, np, torch, natoms, dens, kinds, cut, steps)

    # ---- 5000-atom screening workload: bound vs bound + trained network at the budget ----
    if want("screen5000"):
        from paper_1701_06588_amd import screen
        if os.path.exists(screen.MODEL):
            log("extra: screen5000 ablation")
            w5 = inputs.screen5000()
            dsh5, p5, oo5, off5, tot5 = upload(eng, w5)
            n5 = len(w5.pairs)
            ops5 = list(w5.ops)
            ncand = n5 * len(ops5)
            tau5 = 1e-10 / ncand
            ref5 = torch.empty(tot5, dtype=torch.float64, device=dev)
            got5 = torch.empty(tot5, dtype=torch.float64, device=dev)
            mlp = shg.Mlp(eng, 0)
            mlp.load(screen.MODEL)
            abl = {"workload": "5000 atoms, 60 bohr cube, basis as the 500-atom workload, ordered atom pairs within "
                               "12 bohr, Coulomb and erfc values", "pairs": n5, "candidates": ncand, "tau_blk": tau5,
                   "variants": {}}
            for op in ops5:
                ms_pl, _ = timed(eng, lambda: eng.pairs(dsh5, op, w5.omega[op], p5, oo5, ref5), 3, 1)
                abl["variants"].setdefault("plain", {})[op] = {"ms": round(ms_pl, 4)}
                for vname, model, fl in (("bound", None, 0), ("bound+mlp", mlp, 0),
                                         ("bound, compacting stage", None, shg.PLAN_COMPACT)):
                    pl = shg.Plan(eng, dsh5, op, w5.omega[op], p5, oo5, got5, None, shg.PLAN_PERSISTENT | fl, tau=tau5,
                                  mlp=model)
                    # (a compacting plan builds its queue on the device, in the first two orders only)
                    order = args.tile_order if args.tile_order != "auto" else "round-robin"
                    pl.set_tile_order("alternating" if fl and order == "round-robin" else order)
                    ms_v, _ = timed(eng, pl.execute, 3, 1)
                    bad5, mass5 = compare_chunked(got5, ref5)
                    abl["variants"].setdefault(vname, {})[op] = {
                        "ms": round(ms_v, 4), "skipped": int(pl.skipped().size), "missed_mass": mass5,
                        "kept_bitwise_equal": bad5 == 0}
                    pl.close()
            for d in abl["variants"].values():
                d["blocks_per_s"] = round(ncand / (sum(v["ms"] for v in d.values()) / 1e3), 1)
            mlp.close()
            if args.cpu_sample > 0:
                import oracle
                i5 = np.sort(np.random.default_rng(0).choice(n5, min(20000, n5), replace=False))
                abl["cpu_oracle"] = oracle_rate(
                    lambda: [oracle.pairs(w5.shells, op, w5.omega[op], w5.pairs[i5]) for op in ops5],
                    len(i5) * len(ops5), "blocks/s", f"{len(i5)} random pairs x {len(ops5)} operators, values")
            extra["screen5000_ablation"] = abl
            del ref5, got5
            torch.cuda.empty_cache()
    return extra


if __name__ == "__main__":
    main()
