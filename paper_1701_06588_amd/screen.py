"""Training of the learned prescreener on SHG block magnitudes.

Data: for the five operators (overlap, Coulomb, erfc(0.11 r)/r, erf(0.33 r)/r,
exp(-r^2)), the 12 screening features of every shell pair
(shg_screen_features, derivative-aware bound) and the target log10 of the
largest element of the value block and its three d/dR_a blocks
(shg_block_logmax of blocks the engine evaluates) on the 500-atom workload and
a subset of the molecules workload; split 80/20 by seed (pairs of held-out
atoms / molecules). One model serves every operator (the operator code is a
feature) and both value-only and value+derivative plans (its targets bound
the values too). Training: Adam on the library's own kernels with the
pinball loss at a high quantile (errs towards over-prediction). Calibration:
the margin is the largest under-prediction on the held-out split (plus 0.25);
the training range of every feature is stored so that out-of-range pairs fall
back to the analytic bound.

    python -m paper_1701_06588_amd.screen        # writes prescreen_model.bin
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL = os.path.join(HERE, "prescreen_model.bin")
OPS = ("overlap", "coulomb", "erfc", "erf", "gauss")


def collect(engine, w, ops=OPS, max_pairs=None, seed=0):
    """Features, targets and a held-out mask for workload `w` (device tensors)."""
    import torch
    from paper_1701_06588_amd import shg
    dev = torch.device("cuda")
    pairs_np = w.pairs
    idx = np.arange(len(pairs_np))
    if max_pairs is not None and len(pairs_np) > max_pairs:
        idx = np.sort(np.random.default_rng(seed).choice(len(pairs_np), max_pairs, replace=False))
        pairs_np = pairs_np[idx]
    sub = type(w)(w.name, w.shells, pairs_np, w.ops, w.omega, False)
    off, tot = sub.out_offsets()
    dsh = engine.shells(w.shells)
    pairs = torch.as_tensor(np.ascontiguousarray(pairs_np, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
    dout = torch.empty(max(3 * tot, 1), dtype=torch.float64, device=dev)
    Xs, ys = [], []
    for op in ops:
        engine.pairs(dsh, op, w.omega[op], pairs, oo, out, dout)
        X, _ = shg.screen_features(engine, dsh, op, w.omega[op], pairs, deriv=True)
        y = shg.block_logmax(engine, dsh, pairs, oo, out, dout)
        Xs.append(X.clone())
        ys.append(y.clone())
    # held-out split: pairs whose first atom (or molecule) falls in a fixed 20%
    key = w.shells.atom[pairs_np[:, 0]] if w.mol_of_pair is None else w.mol_of_pair[idx]
    held = (np.asarray(key, np.int64) * 2654435761 % 5) == 0
    held = torch.as_tensor(np.concatenate([held] * len(ops)), device=dev)
    return torch.cat(Xs), torch.cat(ys), held


def train(engine, X, y, held, epochs=25, batch=8192, lr=2e-3, quantile=0.999, seed=0, log=print):
    import torch
    from paper_1701_06588_amd import shg
    Xtr, ytr = X[~held], y[~held]
    Xte, yte = X[held], y[held]
    mean = Xtr.mean(0).cpu().numpy()
    std = Xtr.std(0).cpu().numpy()
    std[std < 1e-6] = 1.0
    lo = Xtr.min(0).values.cpu().numpy()
    hi = Xtr.max(0).values.cpu().numpy()
    mlp = shg.Mlp(engine, seed)
    mlp.set_norm(mean, std, lo, hi)
    mlp.set_scope(OPS, True)
    n = Xtr.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot = 0.0
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            mlp.train_step(Xtr[idx].contiguous(), ytr[idx].contiguous(), lr_ep, quantile, loss)
            tot += float(loss.item()) / batch
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"epoch {ep} mean pinball loss {tot / max(1, n // batch):.4f}")
    pred = torch.empty(Xte.shape[0], dtype=torch.float32, device="cuda")
    inr = torch.empty(Xte.shape[0], dtype=torch.int32, device="cuda")
    mlp.predict(Xte.contiguous(), pred, inr)
    under = (yte - pred)[inr.bool()]
    margin = float(max(0.0, under.max().item()) + 0.25) if under.numel() else 1.0
    mlp.set_margin(margin)
    stats = {"train": int(n), "held_out": int(Xte.shape[0]), "margin": margin,
             "held_mae": float((yte - pred).abs().mean().item()),
             "held_frac_under": float((under > 0).float().mean().item()) if under.numel() else 0.0}
    return mlp, stats


def main(path=MODEL):
    import torch
    from paper_1701_06588_amd import inputs, shg
    t0 = time.time()
    eng = shg.Engine()
    X1, y1, h1 = collect(eng, inputs.five_ops500())
    X2, y2, h2 = collect(eng, inputs.molecules256(n_mol=48), max_pairs=2_000_000)
    X, y, held = torch.cat([X1, X2]), torch.cat([y1, y2]), torch.cat([h1, h2])
    print(f"samples {X.shape[0]} ({time.time() - t0:.1f} s)", flush=True)
    mlp, stats = train(eng, X, y, held, log=lambda m: print(m, flush=True))
    mlp.save(path)
    print(f"saved {path}: {stats} ({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else MODEL)
