"""Autotuner for the launch shapes of the level-batched product.

The product has two launch-shape knobs that change its speed and not its
numbers (up to the summation order of a split sweep):

  mv_split_nodes  a tree level with at most this many nodes runs each node of
                  the up/down sweeps on four wavefronts instead of one;
  mv_xcd_run      the coupling and near products hand nodes to the eight XCDs
                  in runs of this many tree-order neighbours (shared L2).

`tune` builds one handle, then times the product for every candidate value
of one knob at a time (the others held at their best so far), with HIP
events on the stream the product runs on, and returns the fastest shape.
`main` runs it over workloads and writes the table `tuning.json` beside this
file, keyed by a size bin; `Smash(..., tuned=True)` (the default) takes the
launch shape of the nearest bin from it.

    python -m paper_1705_05443_amd.autotune --write [--workloads a,b,...] [--apply p]
"""
from __future__ import annotations

import argparse
import json
import math
import os

KNOBS = {
    "mv_split_nodes": (0, 64, 256, 1024, 4096, 1 << 30),
    "mv_xcd_run": (1, 4, 16, 64),
}
DEFAULTS = {"mv_split_nodes": 1024, "mv_xcd_run": 16}
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def size_bin(n: int, dim: int, adm: str, apply_prec: str, nrhs: int) -> str:
    """Bin of a workload: dimension, admissibility, apply precision, the
    right-hand-side count (1, up to 16, more) and log2 of the point count."""
    rb = 1 if nrhs <= 1 else 16 if nrhs <= 16 else 64
    nb = int(round(math.log2(max(int(n), 2))))
    adm = "strong" if adm in ("strong", "h2") else "weak"
    return "d%d-%s-%s-r%d-n%d" % (dim, adm, apply_prec, rb, nb)


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(n, dim, adm, apply_prec, nrhs, table=None):
    """Launch shape for a workload: the entry of its bin, else of the bin
    with the same dimension, admissibility, precision and right-hand-side
    class whose point count is nearest; None if there is none."""
    table = load_table() if table is None else table
    key = size_bin(n, dim, adm, apply_prec, nrhs)
    if key in table:
        return dict(table[key]["shape"])
    stem, nb = key.rsplit("-n", 1)
    best = None
    for k, v in table.items():
        s, b = k.rsplit("-n", 1)
        if s == stem:
            d = abs(int(b) - int(nb))
            if best is None or d < best[0]:
                best = (d, v["shape"])
    return None if best is None else dict(best[1])


def _time_products(h, Q, reps):
    import torch
    for _ in range(2):
        h.matvec(Q)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        h.matvec(Q)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def tune(x, y=None, nrhs=16, reps=10, seed=0, **kw):
    """Fastest launch shape for the product of this workload.  Returns
    {"shape": {...}, "ms": best product time, "trials": [[knob, value, ms]...]}."""
    import numpy as np
    import torch

    from . import api
    X = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    Y = None if y is None else torch.from_numpy(np.ascontiguousarray(y)).cuda()
    h = api.Smash(X, Y, graphs=False, timing=False, tuned=False, **kw)
    dt = torch.float64 if h.apply_prec == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(seed)
    Q = torch.randn(h.ny, nrhs, generator=g, dtype=torch.float64).to(dt).cuda()
    shape = dict(DEFAULTS)
    trials = []
    best_ms = None
    for knob, values in KNOBS.items():
        best_v = shape[knob]
        for v in values:
            cand = dict(shape)
            cand[knob] = v
            h.set_product_shape(cand["mv_split_nodes"], cand["mv_xcd_run"])
            ms = _time_products(h, Q, reps)
            trials.append([knob, v, ms])
            if best_ms is None or ms < best_ms:
                best_ms, best_v = ms, v
        shape[knob] = best_v
    h.close()
    return {"shape": shape, "ms": best_ms, "trials": trials}


def main(argv=None):
    from . import workloads as W
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workloads", default="h2_2d_log_65536,hss1d_inv_r_2048",
                    help="comma-separated workload names (workloads.CONFIGS)")
    ap.add_argument("--apply", default="", help="override apply precision (f64, f32, bf16)")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--write", action="store_true", help="merge the results into the table")
    ap.add_argument("--out", default=TABLE, help="table to merge into (default tuning.json)")
    args = ap.parse_args(argv)
    table = load_table(args.out)
    for name in args.workloads.split(","):
        cfg = W.CONFIGS[name]
        x, y = W.points(cfg, seed=0)
        apply = args.apply or cfg["apply"]
        kw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"],
                  adm="strong" if cfg["adm"] == 1 else "weak", tol=cfg["tol"], tau=cfg["tau"],
                  root=cfg["root"], apply_prec=apply,
                  eval_prec="f64" if apply == "f64" else "f32")
        if "eps_svd" in cfg:
            kw["eps_svd"] = cfg["eps_svd"]
        nrhs = min(cfg["nrhs"], 64)
        res = tune(x, y, nrhs=nrhs, reps=args.reps, **kw)
        key = size_bin(cfg["n"], cfg["d"], kw["adm"], apply, nrhs)
        res["workload"] = name
        print(key, json.dumps({"shape": res["shape"], "ms": res["ms"]}), flush=True)
        table[key] = res
    if args.write:
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
