#!/usr/bin/env python3
"""Benchmark: one step = SMASH construction + one product, on one MI355X.

Default workload (the paper's H^2 setting of Sec. 6.2 scaled to the 2D
benchmark size): n = 65536 points uniform in the unit square, kernel
log|x-y| (diagonal 0), strong admissibility (tau 0.7), quadtree leaf 64,
8 x 8 Chebyshev interpolation points, RRQR tolerance 1e-8, FP64 build and
product with 16 right-hand sides.  Points and right-hand sides are drawn
from seed 0 and resident in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is points per second through the whole step
(construction + product of 16 vectors).  `roofline` is for the dominant
kernel (measured live with HIP events the library records on the stream it
launches on), `roofline_matvec` for the product, `cpu_baseline` the FP64
oracle on the host cores.
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


def stored_traffic(workload):
    """HBM bytes per launch of the compression kernel and per product, from
    the counter summary under profiles/ -- each None once its source file
    has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", workload + "_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)

    def same(rel, sha):
        with open(os.path.join(ROOT, rel), "rb") as g:
            return hashlib.sha256(g.read()).hexdigest() == sha

    comp = d["bytes_per_launch"] if same(d["source"], d["source_sha256"]) else None
    prod = d.get("product_bytes")
    if prod is not None and not same(d["product_source"], d["product_source_sha256"]):
        prod = None
    return comp, prod


def compr_flops(m, k, c):
    """Algorithmic FP64 flops of compr on one node: the truncated Householder
    QR of the c x m matrix C^T (k reflectors, two flops per multiply-add of
    the dot and of the update) and the triangular solve N = R11^-1 R12."""
    t = np.arange(k)
    qr = np.sum(4.0 * (c - t) * np.maximum(m - t - 1, 0))
    return float(qr + (m - k) * float(k) * k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="h2_2d_log_65536")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target seconds of oracle work for cpu_baseline (0: skip)")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="steps of the plain per-node form timed for comparison (0: skip)")
    ap.add_argument("--skip-evaluated", action="store_true",
                    help="skip the product with coupling blocks evaluated inside it")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times (the "
                         "calibration kernel for the HBM byte counters) and exit")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests in the serving trace (0: skip the serving measurement)")
    ap.add_argument("--serve-rate", type=float, default=40.0, help="mean arrivals per second")
    ap.add_argument("--serve-nmax", type=float, default=2e5,
                    help="largest N of the serving trace (the full stream uses 1e6)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

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
    tdt = torch.float64 if f64 else torch.float32
    X = torch.from_numpy(x).cuda()
    Yd = None if y is None else torch.from_numpy(y).cuda()
    q = W.rhs(n, R, seed=0)
    Q = torch.from_numpy(q.astype(np.float64 if f64 else np.float32)).cuda()
    kw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"],
              adm="strong" if cfg["adm"] == 1 else "weak", tol=cfg["tol"], tau=cfg["tau"],
              root=cfg["root"], apply_prec=cfg["apply"],
              eval_prec="f64" if f64 else "f32")
    if "eps_svd" in cfg:
        kw["eps_svd"] = cfg["eps_svd"]
    torch.cuda.synchronize()

    def step(timing, batched=True):
        h = api.Smash(X, Yd, timing=timing, batched=batched, **kw)
        Z = h.matvec(Q)
        return h, Z

    for _ in range(args.warmup):
        h, Z = step(True)
        h.close()
    torch.cuda.synchronize()

    # ---- timed region: K whole steps -------------------------------------
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h, Z = step(True)
        infos.append(h.info())  # waits for the product; resolves the events
        h.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_step * 1e-3)

    # ---- per-phase device times (HIP events recorded inside the library) ----
    ph = {k: float(np.mean([inf["phase_ms"][k] for inf in infos])) for k in api.PHASES}
    build_ms = float(np.mean([inf["build_ms"] for inf in infos]))

    # ---- one resident handle for sizes, accuracy, product timing ----------
    h = api.Smash(X, Yd, timing=True, **kw)
    inf = h.info()
    rk = h.export("ranks").reshape(-1, 6)
    c = cfg["order"] ** cfg["d"]
    flops = 0.0
    for i in range(1, rk.shape[0]):
        flops += compr_flops(int(rk[i, 0]), int(rk[i, 1]), c + int(rk[i, 4]))
        if not inf["symmetric_reuse"]:
            flops += compr_flops(int(rk[i, 2]), int(rk[i, 3]), c + int(rk[i, 5]))
    e = 8 if f64 else 4
    mv_bytes = (e * R * (n + (n if y is None else len(y)))
                + e * (inf["g_entries_row"] + inf["g_entries_col"])
                + e * (inf["coupling_entries"] + inf["near_entries"])
                + 4 * inf["index_entries"]
                + 2 * e * R * (inf["sum_rank_row"] + inf["sum_rank_col"]))
    reps = 20
    Z = h.matvec(Q)
    torch.cuda.synchronize()
    base = h.info()["phase_ms"]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        Z = h.matvec(Q)
    ev1.record()
    torch.cuda.synchronize()
    mv_eager_ms = ev0.elapsed_time(ev1) / reps
    after = h.info()["phase_ms"]
    mv_ph = {k: (after[k] - base[k]) / reps for k in api.PHASES if k.startswith("mv_")}
    # the resident form: same handle parameters, products replayed from a
    # captured HIP graph (no per-phase events)
    hg = api.Smash(X, Yd, timing=False, **kw)
    Zg = torch.empty_like(Z)
    for _ in range(3):
        hg.matvec(Q, out=Zg)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        hg.matvec(Q, out=Zg)
    ev1.record()
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / reps
    graph_replays = hg.info()["graph_replays"]
    stored_bytes = hg.info()["device_bytes"]
    hg.close()
    # the same product with the coupling blocks evaluated inside it (no
    # stored B; the result is the stored form's bit for bit)
    coupling_evaluated = None
    he = None if args.skip_evaluated else api.Smash(X, Yd, timing=False, coupling="evaluated", **kw)
    if he is not None:
        Ze = torch.empty_like(Z)
        for _ in range(3):
            he.matvec(Q, out=Ze)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            he.matvec(Q, out=Ze)
        ev1.record()
        torch.cuda.synchronize()
        ie = he.info()
        coupling_evaluated = {"matvec_ms": ev0.elapsed_time(ev1) / reps,
                              "device_bytes": int(ie["device_bytes"]),
                              "stored_form_device_bytes": int(stored_bytes),
                              "chunks": int(ie["coupling_chunks"]),
                              "same_as_stored": bool(torch.equal(Ze, Zg))}
        he.close()
    # accuracy against exact rows of A Q
    from oracle import oracle as O
    rows = np.arange(0, n, max(1, n // 512))
    Zc = Z.double().cpu().numpy()
    zr = O.dense_rows(x, x if y is None else y, rows, q, cfg["kernel"])
    err_rows = float(np.linalg.norm(Zc[rows] - zr) / np.linalg.norm(zr))

    compr_ms = ph["compr"]
    dominant = max(ph, key=ph.get)
    tr_comp, tr_prod = stored_traffic(args.workload)
    n_compr = int(infos[0]["phase_calls"]["compr"]) if infos else 0
    roof = {"kernel": "k_compr_w (pivoted Householder QR + Gu-Eisenstat, FP64)", "bound": "alu",
            "achieved": flops / (compr_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "traffic": tr_comp,
            "traffic_note": "HBM bytes per launch (2 x FETCH_SIZE + WRITE_SIZE, calibrated on a "
                            "256 MiB copy), profiles/%s_traffic.md" % args.workload,
            "launches_per_build": n_compr, "ms_per_build": compr_ms,
            "avg_launch_ms": compr_ms / max(n_compr, 1), "algorithmic_flops_per_build": flops}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof_mv = {"kernel": "product (gather, up, coupling, down, near+scatter)", "bound": "hbm",
               "achieved": mv_bytes / (mv_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "traffic": tr_prod, "algorithmic_bytes": mv_bytes, "ms": mv_ms,
               "form": "HIP graph replay (%d replays)" % graph_replays,
               "eager_ms": mv_eager_ms, "eager_phase_ms": mv_ph}
    roof_mv["frac"] = roof_mv["achieved"] / roof_mv["peak"]
    h.close()

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dim": cfg["d"], "kernel": cfg["kernel"],
                   "admissibility": kw["adm"], "leaf": cfg["leaf"], "order": cfg["order"],
                   "tol": cfg["tol"], "tau": cfg["tau"], "nrhs": R, "form": "level-batched"},
        "build_ms": build_ms, "build_points_per_s": n / (build_ms * 1e-3),
        "matvec_ms": mv_ms, "matvec_GBps": roof_mv["achieved"],
        "rel_err_vs_exact_rows": err_rows, "phase_ms": ph, "dominant_phase": dominant,
        "nnodes": int(inf["nnodes"]), "nlevels": int(inf["nlevels"]),
        "roofline": roof, "roofline_matvec": roof_mv,
        "coupling_evaluated": coupling_evaluated,
    }

    # ---- plain per-node form (same kernels, one launch per node) ----------
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            hp, Zp = step(False, batched=False)
            hp.close()
        torch.cuda.synchronize()
        out["plain_form_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / args.plain_steps
        out["speedup_vs_plain_form"] = out["plain_form_ms_per_step"] / ms_step

    # ---- CPU baseline: the FP64 oracle on the host cores --------------------
    if args.cpu_seconds > 0:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        os.environ.setdefault("OMP_NUM_THREADS", str(cores))
        okw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"], adm=cfg["adm"],
                   tol=cfg["tol"], tau=cfg["tau"], root=cfg["root"])
        if "eps_svd" in cfg:
            okw["eps_svd"] = cfg["eps_svd"]
        O.lib()
        reps, t0 = 0, time.perf_counter()
        zo = None
        while True:
            o = O.Oracle(x, y, **okw)
            zo = o.matvec(q)
            del o
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        tc = (time.perf_counter() - t0) / reps
        out["cpu_baseline"] = {"value": n / tc, "unit": "points/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d full steps (build + %d-RHS product) of the same "
                                         "workload, %.2f s each" % (reps, R, tc)}
        out["rel_err_vs_oracle"] = float(np.linalg.norm(Zc - zo) / np.linalg.norm(zo))
    # ---- serving: continuous batching vs one request at a time ------------
    if args.serve_requests > 0:
        from paper_1705_05443_amd import serve
        budget = int(0.8 * torch.cuda.get_device_properties(0).total_memory)

        def serve_run(slots, cap, trace):
            ex = serve.GpuExecutor(slots=slots)
            eng = serve.Engine(ex, budget_bytes=budget, slots=slots, max_batch_rhs=cap)
            done = eng.run(trace)
            st = serve.latency_stats(done)
            st["makespan_s"] = eng.makespan
            st["requests_per_s"] = len(done) / eng.makespan
            st["points_per_s"] = sum(r.rhs.shape[0] for r in done) / eng.makespan
            st["peak_in_flight"] = eng.peak_inflight
            eng.close()
            ex.shutdown()
            return st

        def trace():
            return serve.make_trace(args.serve_requests, rate_hz=args.serve_rate,
                                    n_range=(1e4, args.serve_nmax), seed=1)

        serve_run(4, 64, serve.make_trace(4, rate_hz=100.0, n_range=(1e4, 3e4), seed=99))
        mix = serve_run(4, 64, trace())
        plain = serve_run(1, 1, trace())
        out["serve"] = {
            "trace": "%d requests, Poisson %.0f/s, N log-uniform [1e4, %.0e], dim 2/3, "
                     "uniform/clustered, log r / 1/r / exp(-r), 1-32 FP32 RHS, tol 1e-6, "
                     "30%% products on resident matrices" % (args.serve_requests,
                                                             args.serve_rate, args.serve_nmax),
            "continuous_batching": mix, "plain_one_at_a_time": plain,
            "p99_speedup": plain["p99_ms"] / mix["p99_ms"] if mix.get("p99_ms") else None}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
