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
launch shape of the nearest bin from it.  `order_for` picks the interpolation
order for a tolerance: the smallest whose construction of a sample of the
workload reaches it against exact rows.

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


def exact_rows(x, y, rows, Q, kernel, diag=0.0):
    """Rows of A Q (original order) straight from the kernel's definition, in
    FP64 on the device: 1/|x - y|, log|x - y|, exp(-|x - y|) or 1/(x - y) on
    the line; points that coincide take `diag` (exp(-r): its value 1)."""
    import torch
    X = torch.as_tensor(x, dtype=torch.float64, device="cuda").reshape(len(x), -1)
    Yp = X if y is None else torch.as_tensor(y, dtype=torch.float64,
                                             device="cuda").reshape(len(y), -1)
    Qd = torch.as_tensor(Q, dtype=torch.float64, device="cuda")
    out = []
    for a in range(0, len(rows), 16):
        idx = torch.as_tensor(rows[a:a + 16], device="cuda")
        D = X[idx][:, None, :] - Yp[None, :, :]
        r = torch.sqrt((D * D).sum(-1))
        same = r == 0
        if kernel == "inv_r":
            K = torch.where(same, diag, 1.0 / torch.where(same, 1.0, r))
        elif kernel == "log_r":
            K = torch.where(same, diag, torch.log(torch.where(same, 1.0, r)))
        elif kernel == "exp_r":
            K = torch.exp(-r)
        elif kernel == "cauchy":
            dd = D[..., 0]
            K = torch.where(dd == 0, diag, 1.0 / torch.where(dd == 0, 1.0, dd))
        else:
            raise ValueError("exact rows: kernel %r not supported" % (kernel,))
        out.append(K @ Qd)
    return torch.cat(out).cpu().numpy()


def order_for(x, y=None, *, kernel, tol, orders=range(3, 17), nrhs=4, nrows=256, seed=0,
              **kw):
    """Smallest interpolation order (Chebyshev points per axis, eq. (2.2)) whose
    construction at relative rank tolerance `tol` gives a product within `tol`
    of the exact one, relative Frobenius over `nrows` sampled rows and `nrhs`
    N(0,1) right-hand sides: the order is taken from a measured accuracy, as the
    paper ties the expansion order to the target accuracy (Sec. 6.1; the
    far-field bound (2.9)).  Returns (order, error at that order, [(order,
    error), ...] of the orders tried); if none reaches `tol`, the last one."""
    import numpy as np
    import torch

    from . import api
    X = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    Y = None if y is None else torch.from_numpy(np.ascontiguousarray(y)).cuda()
    ny = len(x) if y is None else len(y)
    q = np.random.default_rng(seed).standard_normal((ny, nrhs))
    Q = torch.from_numpy(q).cuda()
    rows = np.arange(0, len(x), max(1, len(x) // nrows))
    zr = exact_rows(x, y, rows, q, kernel, diag=1.0 if kernel == "exp_r" else 0.0)
    tried = []
    for p in orders:
        h = api.Smash(X, Y, kernel=kernel, order=int(p), tol=tol, apply_prec="f64",
                      graphs=False, tuned=False, **kw)
        z = h.matvec(Q).cpu().numpy()[rows]
        h.close()
        err = float(np.linalg.norm(z - zr) / np.linalg.norm(zr))
        tried.append((int(p), err))
        if err <= tol:
            break
    return tried[-1][0], tried[-1][1], tried


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
