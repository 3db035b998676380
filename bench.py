#!/usr/bin/env python3
"""Benchmark: one step = SMASH construction + one product, on one MI355X.

Headline workload (`--workload`, default h2_3d_inv_r_clusters_1m_p6): the
3D adaptive-tree case at 2^20 points -- 90 % of them from 8 Gaussian
clusters (sigma 0.02) and 10 % uniform in the unit cube -- with kernel
1/|x-y| (diagonal 0), strong admissibility (tau 0.7), octree leaf 128,
6 x 6 x 6 Chebyshev interpolation points and RRQR tolerance 1e-7: the order
at which the product reaches 1e-6 relative error against exact rows of A Q
(5 x 5 x 5 points stop at 4.6e-6).  FP64 construction and FP64 product
with 64 right-hand sides; the coupling blocks (5.5e10 FP64 entries, beyond
one GPU's memory) are evaluated inside each product from their skeleton
index sets.  Points and right-hand sides are drawn from seed 0 and resident
in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  `value` is points per second through the whole step
(construction + product of 64 vectors).  `roofline` is the dominant
kernel's, timed live with the HIP events the library records around each
phase on the stream it launches on.  Further keys: the other workloads as
configured, the plain per-node form, an O(n) series, the oracle on the
host cores (`cpu_baseline`) and the serving loop at three offered loads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "build points/s + matvec GB/s at 1e-6 rel err; serve p50/p99 vs plain form"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def stored_traffic(workload, kernel, calls=1.0):
    """HBM bytes per launch of `kernel` from the counter summary under
    profiles/ (for compr, the bytes of one construction over its `calls`
    launch groups) -- None when absent or when its source file has changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", workload + "_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    ent = d.get("kernels", {}).get(kernel)
    if not ent:
        return None
    with open(os.path.join(ROOT, ent["source"]), "rb") as g:
        if hashlib.sha256(g.read()).hexdigest() != ent["source_sha256"]:
            return None
    if "bytes_per_launch" in ent:
        return ent["bytes_per_launch"]
    return ent["bytes_per_build"] / max(calls, 1.0)


def kwargs_of(cfg):
    kw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"],
              adm="strong" if cfg["adm"] == 1 else "weak", tol=cfg["tol"], tau=cfg["tau"],
              root=cfg["root"], apply_prec=cfg["apply"],
              eval_prec="f64" if cfg["apply"] == "f64" else "f32",
              coupling=cfg.get("coupling", "auto"))
    if "eps_svd" in cfg:
        kw["eps_svd"] = cfg["eps_svd"]
    return kw


def product_bytes(inf, n_x, n_y, R, e):
    """Algorithmic bytes of one product: Q read and Z written once, G of
    both passes, the stored blocks (none for evaluated coupling blocks),
    the index lists, and the skeleton vectors written and read once."""
    blocks = inf["near_entries"] + (0 if inf["coupling_evaluated"] else inf["coupling_entries"])
    return (e * R * (n_x + n_y) + e * (inf["g_entries_row"] + inf["g_entries_col"])
            + e * blocks + 4 * inf["index_entries"]
            + 2 * e * R * (inf["sum_rank_row"] + inf["sum_rank_col"]))


def compr_work(h, inf, c0):
    """FP64 flops of compr per build: sum over nodes and sides of 4 c m k
    (the measure of the cost of the ID, c = basis width), and the exact
    Householder count (sum_t 4 (c - t)(m - t - 1) plus (m - k) k^2 for the
    solve) beside it."""
    rk = h.export("ranks").reshape(-1, 6)[1:].astype(np.float64)
    sides = [(0, 1, 4)] if inf["symmetric_reuse"] else [(0, 1, 4), (2, 3, 5)]
    simple = exact = 0.0
    for mc, kc, sc in sides:
        m, k, c = rk[:, mc], rk[:, kc], c0 + rk[:, sc]
        simple += float(np.sum(4.0 * c * m * k))
        # sum_{t<k} 4 (c - t)(m - t - 1), closed form per node
        t1 = k * (k - 1) / 2.0
        t2 = (k - 1) * k * (2 * k - 1) / 6.0
        exact += float(np.sum(4.0 * (c * (m - 1) * k - (c + m - 1) * t1 + t2)
                              + (m - k) * k * k))
    return simple, exact


def timed_product(h, Q, reps, torch):
    Z = torch.empty((h.nx, Q.shape[1]), dtype=Q.dtype, device=Q.device)
    for _ in range(2):
        h.matvec(Q, out=Z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.matvec(Q, out=Z)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, Z


def kernel_rows(torch, x, y, rows, kernel, pdata=None):
    """Exact FP64 kernel entries K(x[rows], y) on the GPU, straight from the
    kernel's definition: 1/r, log r and exp(-r) (the first two 0 where the
    points coincide), 1/(x - y) on the line, and the Nystrom double layer
    (n_y . (x - y)) / (2 pi r^2) with its per-point diagonal value."""
    X = torch.as_tensor(np.asarray(x, np.float64).reshape(len(x), -1), device="cuda")
    Y = X if y is None else torch.as_tensor(np.asarray(y, np.float64).reshape(len(y), -1),
                                            device="cuda")
    D = X[torch.as_tensor(rows, device="cuda")][:, None, :] - Y[None, :, :]
    r2 = (D * D).sum(-1)
    same = (D == 0).all(-1)
    if kernel == "inv_r":
        K = torch.where(same, 0.0, 1.0 / torch.sqrt(r2))
    elif kernel == "log_r":
        K = torch.where(same, 0.0, torch.log(torch.sqrt(r2)))
    elif kernel == "exp_r":
        K = torch.exp(-torch.sqrt(r2))
    elif kernel == "cauchy":
        K = 1.0 / D[..., 0]
    elif kernel == "double_layer":
        pd = torch.as_tensor(np.asarray(pdata, np.float64).reshape(-1, 3), device="cuda")
        proj = (D * pd[None, :, :2]).sum(-1)
        K = torch.where(same, pd[torch.as_tensor(rows, device="cuda"), 2][:, None],
                        proj / (2.0 * np.pi * r2))
    else:
        raise ValueError(kernel)
    return K


def exact_rows(torch, x, y, rows, q, kernel, chunk=16, nb=256):
    """Rows of A Q for the given original row indices, in FP64.  The long
    inner dimension is split into nb batched products whose results are
    summed (a product of 16 rows against 10^6 x 64 is one output tile and
    would otherwise run on a single workgroup)."""
    Q = torch.as_tensor(np.asarray(q, np.float64).reshape(q.shape[0], -1), device="cuda")
    n, R = Q.shape
    L = -(-n // nb)
    Qb = torch.zeros((nb * L, R), dtype=torch.float64, device="cuda")
    Qb[:n] = Q
    Qb = Qb.view(nb, L, R)
    out = []
    for a in range(0, len(rows), chunk):
        K = kernel_rows(torch, x, y, rows[a:a + chunk], kernel)
        Kb = torch.zeros((K.shape[0], nb * L), dtype=torch.float64, device="cuda")
        Kb[:, :n] = K
        Kb = Kb.view(K.shape[0], nb, L).transpose(0, 1).contiguous()
        out.append(torch.bmm(Kb, Qb).sum(0))
    return torch.cat(out).cpu().numpy()


def rows_error(Z, x, y, q, kernel, n, nrows=512):
    import torch
    rows = np.arange(0, n, max(1, n // nrows))
    zr = exact_rows(torch, x, y, rows, q, kernel)
    Zc = Z.double().cpu().numpy()
    return float(np.linalg.norm(Zc[rows] - zr) / np.linalg.norm(zr))


def one_workload(name, torch, api, W, reps=5, nrhs=None, apply=None, n=None):
    """One construction and timed products of a workload: build and product
    times, phase times, error against exact rows."""
    cfg = dict(W.CONFIGS[name])
    if apply:
        cfg["apply"] = apply
    x, y = W.points(cfg, seed=0, n=n)
    nn = len(x)
    R = nrhs or cfg["nrhs"]
    f64 = cfg["apply"] == "f64"
    X = torch.from_numpy(x).cuda()
    Yd = None if y is None else torch.from_numpy(y).cuda()
    q = W.rhs(len(x if y is None else y), R, seed=0)
    if not f64:
        q = q.astype(np.float32).astype(np.float64)
    Q = torch.from_numpy(q).to(torch.float64 if f64 else torch.float32).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = api.Smash(X, Yd, timing=True, **kwargs_of(cfg))
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    inf = h.info()
    h.close()
    hg = api.Smash(X, Yd, timing=False, **kwargs_of(cfg))
    ms, Z = timed_product(hg, Q, reps, torch)
    ig = hg.info()
    e = 8 if f64 else 4
    mvb = product_bytes(ig, nn, len(x if y is None else y), R, e)
    out = {"n": nn, "nrhs": R, "apply": cfg["apply"], "order": cfg["order"], "tol": cfg["tol"],
           "build_ms": wall, "build_points_per_s": nn / (wall * 1e-3),
           "build_phase_ms": {k: v for k, v in inf["phase_ms"].items() if v > 0},
           "matvec_ms": ms, "matvec_GBps": mvb / (ms * 1e-3) / 1e9,
           "coupling_evaluated": bool(ig["coupling_evaluated"]),
           "device_GB": ig["device_bytes"] / 1e9,
           "rel_err_vs_exact_rows": rows_error(Z, x, y, q, cfg["kernel"], nn)}
    hg.close()
    del X, Yd, Q, Z
    torch.cuda.empty_cache()
    return out


def cauchy_like_bench(torch, api, W, n=1 << 20, p=2, nrhs=16, reps=5):
    """Sec. 6.3's Cauchy-like matrix (eq. (6.1), p generator columns of
    U(0,1) entries) on the interlaced points of eq. (6.3): the HSS
    construction of the Cauchy matrix (tau 0.6, leaf 50, eps_SVD 1e-9, as in
    Sec. 6.3; 16 Chebyshev points and tol 1e-8 in place of the Taylor basis),
    the Cauchy-like product by eq. (6.2) against the plain product of the
    same handle, and its error against exact rows of (6.1)."""
    x, y = W.interlaced_pair(n, seed=0)
    w, v = W.cauchy_like_generators(n, n, p, seed=0)
    q = W.rhs(n, nrhs, seed=0)
    X, Yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    Q, Wd, Vd = (torch.from_numpy(a).cuda() for a in (q, w, v))
    kw = dict(kernel="cauchy", leaf=50, order=16, adm="weak", tol=1e-8, eps_svd=1e-9, tau=0.6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = api.Smash(X, Yd, timing=True, **kw)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    inf = h.info()
    h.close()
    hg = api.Smash(X, Yd, **kw)
    Z = torch.empty((n, nrhs), dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        hg.matvec_cauchy_like(Q, Wd, Vd, out=Z)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        hg.matvec_cauchy_like(Q, Wd, Vd, out=Z)
    ev[1].record()
    Zp = hg.matvec(Q)
    ev[2].record()
    for _ in range(reps):
        hg.matvec(Q, out=Zp)
    ev[3].record()
    torch.cuda.synchronize()
    rows = np.arange(0, n, n // 256)
    zr = sum(w[rows, l:l + 1] * exact_rows(torch, x, y, rows, v[:, l:l + 1] * q, "cauchy")
             for l in range(p))
    err = float(np.linalg.norm(Z.cpu().numpy()[rows] - zr) / np.linalg.norm(zr))
    out = {"n": n, "p": p, "nrhs": nrhs, "points": "eq. (6.3), shift 1e-7", "build_ms": wall,
           "build_phase_ms": {k: v for k, v in inf["phase_ms"].items() if v > 0},
           "cauchy_like_product_ms": ev[0].elapsed_time(ev[1]) / reps,
           "plain_product_ms": ev[2].elapsed_time(ev[3]) / reps,
           "rel_err_vs_exact_rows": err, "max_rank": int(inf["max_rank_row"])}
    hg.close()
    del X, Yd, Q, Wd, Vd, Z, Zp
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="h2_3d_inv_r_clusters_1m_p6")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target seconds of oracle work for cpu_baseline (0: skip)")
    ap.add_argument("--cpu-n", type=int, default=1 << 15,
                    help="points of the oracle's sample of the workload")
    ap.add_argument("--plain-n", type=int, default=1 << 16,
                    help="points at which the plain per-node form is compared (0: skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also time the other workloads and the O(n) series (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times (the "
                         "calibration kernel for the HBM byte counters) and exit")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests per offered load in the serving trace (0: skip)")
    ap.add_argument("--serve-nmax", type=float, default=1e6,
                    help="largest N of the serving trace")
    ap.add_argument("--serve-only", default="",
                    help="only run the serving section and write its results as JSON to "
                         "this path (the main run starts itself this way)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.serve_only:
        res = serve_bench(args, torch)
        with open(args.serve_only, "w") as f:
            json.dump(res, f)
        return

    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                          "launches": 5}), flush=True)
        return

    from paper_1705_05443_amd import api
    from paper_1705_05443_amd import workloads as W

    cfg = W.CONFIGS[args.workload]
    x, y = W.points(cfg, seed=0)
    n = cfg["n"]
    R = cfg["nrhs"]
    f64 = cfg["apply"] == "f64"
    X = torch.from_numpy(x).cuda()
    Yd = None if y is None else torch.from_numpy(y).cuda()
    q = W.rhs(n, R, seed=0)
    if not f64:
        q = q.astype(np.float32).astype(np.float64)
    Q = torch.from_numpy(q).to(torch.float64 if f64 else torch.float32).cuda()
    kw = kwargs_of(cfg)
    torch.cuda.synchronize()

    def step(timing=True, batched=True, XX=X, QQ=Q):
        h = api.Smash(XX, None if y is None else Yd, timing=timing, batched=batched, **kw)
        Z = h.matvec(QQ)
        return h, Z

    print("warmup", flush=True)
    for _ in range(args.warmup):
        h, Z = step()
        h.close()
    torch.cuda.synchronize()

    # ---- timed region: K whole steps -------------------------------------
    print("timed steps", flush=True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h, Z = step()
        infos.append(h.info())  # waits for the product; resolves the events
        h.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_step * 1e-3)

    # ---- per-phase device times (HIP events recorded inside the library) ----
    ph = {k: float(np.mean([inf["phase_ms"][k] for inf in infos])) for k in api.PHASES}
    calls = {k: float(np.mean([inf["phase_calls"][k] for inf in infos])) for k in api.PHASES}
    build_ms = float(np.mean([inf["build_ms"] for inf in infos]))

    # ---- one resident handle: sizes, accuracy, product timing -------------
    h = api.Smash(X, Yd, timing=False, **kw)
    inf = h.info()
    c0 = cfg["order"] ** cfg["d"]
    compr_simple, compr_exact = compr_work(h, inf, c0)
    e = 8 if f64 else 4
    mv_ms, Z = timed_product(h, Q, 5, torch)
    mv_bytes = product_bytes(inf, n, n if y is None else len(y), R, e)
    coupling_flops = 2.0 * R * inf["coupling_entries"]
    mv_flops = 2.0 * R * (inf["coupling_entries"] + inf["near_entries"]
                          + 2 * (inf["g_entries_row"] + inf["g_entries_col"]))
    print("exact rows", flush=True)
    err_rows = rows_error(Z, x, y, q, cfg["kernel"], n)
    storage = {k: inf[k] for k in ("bytes_dense", "bytes_hss0", "bytes_smash", "device_bytes")}
    h.close()

    # ---- roofline of the dominant kernel ----------------------------------
    dominant = max(ph, key=ph.get)

    def roofline_of(phase):
        """Roofline of the kernel behind a phase: compr (pivoted Householder QR
        with the Gu-Eisenstat swaps, FP64 ALU) or the coupling contraction
        (matrix cores), else an HBM-bound entry without a figure."""
        if phase == "compr":
            r = {"kernel": "k_compr_dq / k_compr_w / k_compr_s (pivoted Householder QR + "
                           "Gu-Eisenstat, FP64)",
                 "bound": "alu", "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "work": "sum over nodes of 4 c m k FP64 flops", "work_per_build": compr_simple,
                 "exact_householder_flops_per_build": compr_exact}
            r["achieved"] = compr_simple / (ph["compr"] * 1e-3) / 1e12
            r["achieved_exact_count"] = compr_exact / (ph["compr"] * 1e-3) / 1e12
            r["traffic"] = stored_traffic(args.workload, "compr", calls["compr"])
        elif phase == "mv_coupling":
            fp = FP64_PEAK_TFLOPS if f64 else FP32_PEAK_TFLOPS
            r = {"kernel": "k_mv_coupling_eval (blocks evaluated in the contraction, %s MFMA)"
                           % ("FP64" if f64 else "FP32") if inf["coupling_evaluated"]
                 else "k_mv_coupling", "bound": "mfma", "peak": fp, "unit": "TFLOP/s",
                 "work": "2 R sum_L k_i k_j flops", "work_per_launch": coupling_flops}
            r["achieved"] = coupling_flops / (ph["mv_coupling"] / max(calls["mv_coupling"], 1)
                                              * 1e-3) / 1e12
            r["traffic"] = stored_traffic(args.workload, "mv_coupling")
        else:
            r = {"kernel": phase, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "achieved": None, "traffic": None}
        r["ms_per_step"] = ph[phase]
        r["launches_per_step"] = calls[phase]
        r["avg_launch_ms"] = ph[phase] / max(calls[phase], 1)
        r["frac"] = r["achieved"] / r["peak"] if r.get("achieved") else None
        return r

    roof = roofline_of(dominant)
    roof_mv = {"kernel": "product (gather, up, coupling, down, near+scatter)", "ms": mv_ms,
               "algorithmic_bytes": mv_bytes, "GBps": mv_bytes / (mv_ms * 1e-3) / 1e9,
               "hbm_frac": mv_bytes / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "flops": mv_flops, "TFLOPs": mv_flops / (mv_ms * 1e-3) / 1e12}

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dim": cfg["d"], "kernel": cfg["kernel"],
                   "points": cfg["kind"], "admissibility": kw["adm"], "leaf": cfg["leaf"],
                   "order": cfg["order"], "tol": cfg["tol"], "tau": cfg["tau"], "nrhs": R,
                   "coupling": cfg.get("coupling", "auto"), "form": "level-batched"},
        "build_ms": build_ms, "build_points_per_s": n / (build_ms * 1e-3),
        "matvec_ms": mv_ms, "matvec_GBps": roof_mv["GBps"],
        "rel_err_vs_exact_rows": err_rows, "phase_ms": ph, "phase_calls": calls,
        "dominant_phase": dominant, "nnodes": int(inf["nnodes"]), "nlevels": int(inf["nlevels"]),
        "roofline": roof, "roofline_compr": roofline_of("compr"),
        "roofline_coupling": roofline_of("mv_coupling"),
        "roofline_matvec": roof_mv, "storage_bytes": storage,
    }
    print("headline %.1f ms/step" % ms_step, flush=True)

    # ---- plain per-node form (same kernels, one launch per node) ----------
    if args.plain_n > 0:
        print("plain form", flush=True)
        xs = W.points(cfg, seed=0, n=args.plain_n)[0] if y is None else None
        if xs is not None:
            Xs = torch.from_numpy(xs).cuda()
            Qs = Q[:args.plain_n].contiguous()
            res = {}
            for form, bt in (("level_batched", True), ("plain_per_node", False)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                hs, _ = step(False, bt, Xs, Qs)
                torch.cuda.synchronize()
                res[form + "_ms_per_step"] = (time.perf_counter() - t0) * 1e3
                hs.close()
            res["n"] = args.plain_n
            res["speedup"] = res["plain_per_node_ms_per_step"] / res["level_batched_ms_per_step"]
            out["plain_form"] = res
            del Xs, Qs

    # ---- the other workloads as configured, and the O(n) series ------------
    if args.extras:
        print("extras", flush=True)
        ex = {}
        ex["h2_2d_log_65536"] = one_workload("h2_2d_log_65536", torch, api, W, reps=20)
        ex["h2_3d_inv_r_clusters_1m (5^3 points, FP32 apply)"] = one_workload(
            "h2_3d_inv_r_clusters_1m", torch, api, W, reps=3)
        ex["hss1d_inv_r_2048"] = one_workload("hss1d_inv_r_2048", torch, api, W, reps=20)
        ex["hss1d_cauchy_1m (FP32 apply)"] = one_workload("hss1d_cauchy_1m", torch, api, W,
                                                          reps=3)
        ex["hss1d_cauchy_1m (BF16 apply)"] = one_workload("hss1d_cauchy_1m", torch, api, W,
                                                          reps=3, apply="bf16")
        out["workloads"] = ex
        print("double layer", flush=True)
        out["double_layer"] = double_layer_bench(torch, api, W)
        print("Cauchy-like", flush=True)
        out["cauchy_like"] = cauchy_like_bench(torch, api, W)
        print("O(n) series", flush=True)
        ser = []
        for lg in range(14, 21):
            nn = 1 << lg
            xs = W.points(cfg, seed=0, n=nn)[0]
            Xs = torch.from_numpy(xs).cuda()
            Qs = Q[:nn].contiguous()
            hs, _ = step(False, True, Xs, Qs)
            hs.close()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hs = api.Smash(Xs, None, timing=False, **kw)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) * 1e3
            tm, _ = timed_product(hs, Qs, 2, torch)
            hs.close()
            ser.append({"n": nn, "build_ms": tb, "matvec_ms": tm,
                        "build_us_per_point": tb * 1e3 / nn, "matvec_ns_per_point": tm * 1e6 / nn})
            del Xs, Qs
        out["on_series"] = ser

    # ---- CPU baseline: the FP64 oracle on the host cores --------------------
    if args.cpu_seconds > 0:
        print("cpu baseline", flush=True)
        from oracle import oracle as O
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        os.environ.setdefault("OMP_NUM_THREADS", str(cores))
        okw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"], adm=cfg["adm"],
                   tol=cfg["tol"], tau=cfg["tau"], root=cfg["root"])
        if "eps_svd" in cfg:
            okw["eps_svd"] = cfg["eps_svd"]
        O.lib()
        nc = min(args.cpu_n, n)
        xs = W.points(cfg, seed=0, n=nc)[0]
        qs = q[:nc]
        reps, t0 = 0, time.perf_counter()
        while True:
            o = O.Oracle(xs, None, **okw)
            o.matvec(qs)
            del o
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        tc = (time.perf_counter() - t0) / reps
        out["cpu_baseline"] = {"value": nc / tc, "unit": "points/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d full steps (build + %d-RHS product) of the workload's "
                                         "point distribution and parameters at n = %d, %.2f s "
                                         "each" % (reps, R, nc, tc)}
    # ---- serving: continuous batching at three offered loads --------------
    if args.serve_requests > 0:
        print("serving", flush=True)
        out["serve"] = serve_in_child(args, torch, api)
    print(json.dumps(out), flush=True)


def serve_in_child(args, torch, api):
    """The serving section in a process of its own (it runs several streams
    of constructions and products at once): its results, or, if it fails,
    its exit status, without ending the measurement above."""
    import subprocess
    import tempfile
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    api.trim()
    fd, path = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--serve-only", path,
           "--serve-requests", str(args.serve_requests), "--serve-nmax", repr(args.serve_nmax)]
    try:
        rc = subprocess.run(cmd, timeout=1500).returncode
        if rc != 0:
            return {"error": "serving process exited with status %d" % rc}
        with open(path) as f:
            return json.load(f)
    except subprocess.TimeoutExpired:
        return {"error": "serving process exceeded 1500 s"}
    finally:
        os.unlink(path)


def double_layer_bench(torch, api, W):
    """Sec. 6.4's HSS constructions of the Nystrom double-layer matrix at the
    size of Table 6.6 (n = 10240) on both curves, at the tolerances of that
    table: build time (one construction, phase timers on), ||A - A_hat||_max
    against the dense matrix (Tables 6.3-6.4), the storage comparison of
    Table 6.6 (in MiB: the dense matrix is the table's 800), and the skeleton
    sizes of the root's children (the size(B_i) of Table 6.5)."""
    res = {}
    n = 10240
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    for curve in ("ram_head", "sunflower"):
        pts, data = W.curve(curve, n)
        P, D = torch.from_numpy(pts).cuda(), torch.from_numpy(data).cuda()
        for tol, eps in ((1e-4, 1e-5), (1e-10, 1e-11)):
            kw = dict(kernel="double_layer", leaf=50, order=5, adm="weak", tol=tol,
                      eps_svd=eps, tau=0.6)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = api.Smash(P, point_data=D, timing=True, **kw)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) * 1e3
            phases = h.info()["phase_ms"]
            Ah = h.matvec(eye)
            err = 0.0
            for a in range(0, n, 256):  # A_hat = A_hat I against A, in row blocks
                rows = np.arange(a, min(n, a + 256))
                Kt = kernel_rows(torch, pts, None, rows, "double_layer", data)
                err = max(err, float((Kt - Ah[rows[0]:rows[-1] + 1]).abs().max()))
            inf = h.info()
            rk = h.export("ranks").reshape(-1, 6)
            nodes = h.export("nodes").reshape(-1, 8)
            kids = [int(nodes[0, 2]), int(nodes[0, 2]) + 1]
            key = "%s tol %.0e eps_svd %.0e" % (curve, tol, eps)
            res[key] = {
                "n": n, "build_ms": tb, "max_abs_err": err,
                "storage_MiB": {"dense": inf["bytes_dense"] / 2**20,
                                "hss0": inf["bytes_hss0"] / 2**20,
                                "smash": inf["bytes_smash"] / 2**20},
                "root_children_skeletons_row_col": [[int(rk[c, 1]), int(rk[c, 3])] for c in kids],
                "phase_ms": {k: v for k, v in phases.items() if v > 0},
                "nlevels": int(inf["nlevels"])}
            h.close()
            del Ah
            print("double layer %s: build %.1f ms, max err %.2e" % (key, tb, err), flush=True)
    return res


def serve_bench(args, torch):
    """The serving stream: construct-and-apply requests (N log-uniform in
    [1e4, nmax], dim 2 or 3, uniform or clustered, log r / 1/r / exp(-r),
    1-32 FP32 right-hand sides, tol 1e-6), 30 % products on resident
    matrices.  The capacity of the plain serial form (one request at a time)
    is measured first; then the continuous-batching engine and the plain
    form run the same Poisson trace at 0.5, 0.8 and 1.0 times it."""
    from paper_1705_05443_amd import api, serve
    # the earlier sections' cached memory goes back to the device; the
    # handles then take theirs from torch's caching allocator, which also
    # holds the vectors (one allocator, which frees its cache and retries
    # before it fails)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    api.trim()
    free, total = torch.cuda.mem_get_info()
    budget = int(min(0.8 * total, 0.85 * free))
    # torch's allocator (handles and vectors, its cache of freed blocks
    # included) stays within this share of the device; the rest is left to
    # the runtime (scratch memory of the kernels that spill, queues, events)
    fraction = min(0.85, 0.9 * free / total)
    torch.cuda.reset_peak_memory_stats()

    def run(slots, cap, trace, keep=None):
        ex = serve.GpuExecutor(slots=slots, allocator="torch", memory_fraction=fraction)
        eng = serve.Engine(ex, budget_bytes=budget, slots=slots, max_batch_rhs=cap)
        done = eng.run(trace)
        st = serve.latency_stats(done)
        st["makespan_s"] = eng.makespan
        st["requests_per_s"] = len(done) / eng.makespan
        st["points_per_s"] = sum(r.rhs.shape[0] for r in done) / eng.makespan
        st["peak_in_flight"] = eng.peak_inflight
        reasons = {}
        for r in done:
            if r.error is not None:
                reasons[r.error] = reasons.get(r.error, 0) + 1
        st["failure_reasons"] = reasons
        eng.close()
        ex.shutdown()
        if keep is not None:
            keep.extend(done)
        return st

    def trace(num, rate):
        # FP32 right-hand sides, products in FP64 (FP32 products of 1e6
        # points stay near 1.6e-6 from exact rows, above the tolerance)
        return serve.make_trace(num, rate_hz=rate, n_range=(1e4, args.serve_nmax), seed=1,
                                apply_prec="f64")

    nreq = args.serve_requests
    run(4, 64, serve.make_trace(4, rate_hz=100.0, n_range=(1e4, 3e4), seed=99,
                                apply_prec="f64"))  # warm-up
    print("serve warm-up done", flush=True)
    # capacity of the plain form: the whole trace offered at once
    cap = run(1, 1, trace(nreq, 1e6))
    capacity = cap["requests_per_s"]
    print("serve capacity %.2f requests/s" % capacity, flush=True)
    res = {"trace": "%d requests per load, N log-uniform [1e4, %.0e], dim 2/3, "
                    "uniform/clustered, log r / 1/r / exp(-r), 1-32 FP32 RHS (FP64 products), "
                    "tol 1e-6, Chebyshev points per axis %s by dimension, 30%% products on "
                    "resident matrices, Poisson arrivals" % (nreq, args.serve_nmax,
                                                             serve.SERVE_ORDER),
           "plain_capacity_requests_per_s": capacity, "budget_GB": budget / 1e9,
           "torch_memory_fraction": fraction, "loads": {}}
    for load in (0.5, 0.8, 1.0):
        rate = load * capacity
        kept = [] if load == 1.0 else None
        # two worker streams: with four, concurrent 10^6-point constructions
        # contend and every latency percentile was worse than with two
        mix = run(2, 64, trace(nreq, rate), kept)
        plain = run(1, 1, trace(nreq, rate))
        res["loads"]["%.1f" % load] = {
            "rate_per_s": rate, "continuous_batching": mix, "plain_one_at_a_time": plain,
            "p99_speedup": plain["p99_ms"] / mix["p99_ms"] if mix.get("p99_ms") else None}
        print("serve load %.1f done" % load, flush=True)
    # accuracy of served results: sampled rows of the largest and smallest
    # constructions against exact rows of A Q
    builds = sorted((r for r in kept if r.points is not None and r.error is None),
                    key=lambda r: r.points.shape[0])
    errs = []
    for r in builds[:2] + builds[-3:]:
        nn = r.points.shape[0]
        rows = np.arange(0, nn, max(1, nn // 64))
        zr = exact_rows(torch, r.points, None, rows,
                        r.rhs.astype(np.float32).astype(np.float64), r.params["kernel"])
        errs.append({"n": nn, "dim": r.points.shape[1], "kernel": r.params["kernel"],
                     "rel_err_vs_exact_rows":
                         float(np.linalg.norm(r.result[rows] - zr) / np.linalg.norm(zr))})
    res["accuracy"] = errs
    res["torch_peak_reserved_GB"] = torch.cuda.max_memory_reserved() / 1e9
    return res


if __name__ == "__main__":
    main()
