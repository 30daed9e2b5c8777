"""Autotuning of the per-class tile shapes (driver around shg_autotune).

``python -m paper_1701_06588_amd.tune`` tunes every operator, with and without
derivatives, on the 500-atom workload and writes ``tune_cache.json`` next to
the library; ``apply_cache(engine)`` loads it (entries of other GPU
architectures are ignored by the library)."""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")


def apply_cache(engine, path: str = CACHE) -> int:
    if not os.path.exists(path):
        return 0
    return engine.tuning_load(path)


def tune(path: str = CACHE, reps: int = 3) -> None:
    import numpy as np
    import torch
    from paper_1701_06588_amd import inputs, shg
    w = inputs.five_ops500()
    eng = shg.Engine()
    dev = torch.device("cuda")
    dsh = eng.shells(w.shells)
    off, tot = w.out_offsets()
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    oo = torch.as_tensor(off, device=dev)
    out = torch.empty(tot, dtype=torch.float64, device=dev)
    dout = torch.empty(3 * tot, dtype=torch.float64, device=dev)
    for op in inputs.FIVE_OPS:
        for deriv in (False, True):
            eng.autotune(dsh, op, w.omega[op], pairs, oo, out, dout if deriv else None, reps)
            print(f"tuned {op} deriv={deriv}", flush=True)
    eng.tuning_save(path)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    tune(sys.argv[1] if len(sys.argv) > 1 else CACHE)
