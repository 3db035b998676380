"""Serving loop: continuous batching of construct-and-apply requests.

Requests arrive over time (a trace of arrival times).  Each asks for the
product of a kernel matrix with 1-32 right-hand sides; the matrix is either
built from the request's points (a construction) or one already resident
on the device (a product only).  The engine

  * takes the waiting requests shortest estimated work first (less the
    time they have waited, so none starves), and keeps at most one large
    construction in flight;
  * admits a construction when a worker slot is free and its device
    footprint fits the memory budget beside everything resident or in
    flight -- while it runs, the footprint is the library's upper estimate
    (smash_estimate_footprint) scaled by the largest ratio of a
    construction's peak device bytes (temporaries included, from
    smash_info) to the estimate seen so far (seeded from the autotuner
    table), with a margin; once built, the matrix holds its resident bytes;
  * evicts idle resident matrices, least recently used first, to make room,
    and builds an evicted matrix again from its points when a product on
    it arrives later;
  * admits a construction whose stored form exceeds the whole budget with
    its coupling blocks evaluated inside each product instead
    (SMASH_COUPLING_EVALUATED: the same results, no O(sum k_i k_j) storage,
    slower products);
  * merges the waiting product requests of one resident matrix into a
    single multi-right-hand-side product (one pass over its blocks);
  * runs admitted work on worker threads, one HIP stream each, so builds
    and products of different requests overlap on the device, and admits
    new requests as soon as slots and memory free up;
  * reports per-request latency (completion - arrival) percentiles beside
    throughput.

The scheduler is independent of the device: an executor runs the work.
`GpuExecutor` runs it through the C library; tests drive the same
scheduler with a host-only executor.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


SMASH_E_OOM = -3  # the library's out-of-memory code


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the trace
    matrix: str                    # id of the matrix (resident-cache key)
    rhs: np.ndarray                # (n, nrhs)
    points: np.ndarray | None = None  # (n, dim) FP64 for a construction, else None
    params: dict = field(default_factory=dict)  # kernel, leaf, order, adm, tol, apply_prec
    # filled by the engine
    admitted: float = math.nan
    done: float = math.nan
    result: np.ndarray | None = None
    error: str | None = None
    batch: int = 0                 # requests served by the same product launch
    retries: int = 0               # constructions re-queued after running out of memory


@dataclass
class Resident:
    matrix: str
    handle: object
    bytes: int
    busy: bool = False
    last_use: float = 0.0


class Engine:
    def __init__(self, executor, budget_bytes: int, slots: int = 4, margin: float = 1.15,
                 ratio: float | None = None, max_batch_rhs: int = 64, lookahead: int = 8,
                 allow_evaluated: bool = True, shortest_first: bool = True,
                 heavy_points: int = 200_000, max_heavy: int = 1, age_weight: float = 1.0,
                 oom_retries: int = 2):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.margin = margin
        self.ratios = {} if ratio is None else {None: ratio}  # resident / estimated bytes
        self.peak_ratios = {}  # a construction's peak (temporaries included) / estimated bytes
        self.max_batch_rhs = max_batch_rhs
        self.lookahead = lookahead
        self.allow_evaluated = allow_evaluated
        # admission order and the limit on large constructions in flight
        self.shortest_first = shortest_first
        self.heavy_points = heavy_points
        self.max_heavy = max_heavy
        self.age_weight = age_weight
        # a construction that fails for want of memory (SMASH_E_OOM: the
        # reservation was met but the allocator could not place a block) is
        # queued again, up to oom_retries times, and runs when memory frees up
        self.oom_retries = oom_retries
        self.requeue = []
        self.resident: dict[str, Resident] = collections.OrderedDict()
        self.sources = {}             # matrix -> (points, params) it was built from
        self.inflight = []            # (future, kind, requests, reserved bytes, matrix)
        self.reserved = 0             # bytes of resident matrices + builds in flight
        self.peak_reserved = 0
        self.peak_inflight = 0
        self.log = []

    # ---- memory model ---------------------------------------------------
    @staticmethod
    def _evaluated(req):
        return req.params.get("coupling") == "evaluated"

    @staticmethod
    def _cls(req, evaluated=False):
        return None if req.points is None else (req.points.shape[1], bool(evaluated))

    def _need(self, req, evaluated=False):
        """Bytes reserved while a construction runs (stored or evaluated
        coupling blocks): the estimate times the largest ratio of a
        construction's peak device bytes (its temporaries included) to the
        estimate seen for its dimension and form -- before any, the resident
        ratio, the executor's prior, else 1 -- with the margin, never above
        1.  Once built, the matrix holds its resident bytes only."""
        est = self.ex.estimate(req, evaluated=evaluated)
        c = self._cls(req, evaluated)
        r = self.peak_ratios.get(c, self.ratios.get(c, self.ratios.get(None)))
        if r is None:
            r = self.ex.prior_ratio(req)
        return int(est * min(1.0, r * self.margin))

    def _evict_for(self, need, wanted=()):
        """Evict idle resident matrices (LRU) until `need` more bytes fit,
        never one in `wanted` (matrices that waiting product requests name:
        evicting it would fail them)."""
        for m in list(self.resident):
            if self.reserved + need <= self.budget:
                break
            res = self.resident[m]
            if res.busy or m in wanted:
                continue
            self.ex.release(res.handle)
            self.reserved -= res.bytes
            del self.resident[m]
            self.log.append(("evict", m))
        return self.reserved + need <= self.budget

    # ---- main loop ------------------------------------------------------
    def run(self, requests, realtime=True, poll=0.0005):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        i = 0
        done = []
        building = set()  # matrices whose construction is in flight
        while i < len(reqs) or pending or self.inflight:
            t = now()
            while i < len(reqs) and (reqs[i].arrival <= t or not realtime):
                pending.append(reqs[i])
                i += 1
            progressed = self._reap(done, building, now)
            while self.requeue:
                pending.appendleft(self.requeue.pop())
            progressed |= self._admit(pending, building, now, done)
            if not progressed:
                if self.inflight or pending:
                    time.sleep(poll)
                elif i < len(reqs) and realtime:
                    time.sleep(max(0.0, min(0.01, reqs[i].arrival - now())))
        self.makespan = now()
        return done

    def _reap(self, done, building, now):
        progressed = False
        keep = []
        for fut, kind, group, resv, m in self.inflight:
            if not fut.done():
                keep.append((fut, kind, group, resv, m))
                continue
            progressed = True
            t = now()
            try:
                out = fut.result()
            except Exception as e:  # a failed request frees what it held
                if (kind == "build" and getattr(e, "code", None) == SMASH_E_OOM
                        and all(r.retries < self.oom_retries for r in group)):
                    self.reserved -= resv
                    building.discard(m)
                    for r in group:
                        r.retries += 1
                    self.requeue.extend(group)
                    self.log.append(("requeue", m))
                    continue
                for r in group:
                    r.error, r.done = str(e), t
                    done.append(r)
                if kind == "build":
                    self.reserved -= resv
                    building.discard(m)
                else:
                    self.resident[m].busy = False
                continue
            if kind == "build":
                # (handle, resident bytes, results[, peak bytes of the build])
                handle, nbytes, results = out[:3]
                peak = out[3] if len(out) > 3 else nbytes
                building.discard(m)
                ev = self._evaluated(group[0])
                est = self.ex.estimate(group[0], evaluated=ev)
                if est > 0:
                    c = self._cls(group[0], ev)
                    self.ratios[c] = max(self.ratios.get(c, 0.0), nbytes / est)
                    self.peak_ratios[c] = max(self.peak_ratios.get(c, 0.0),
                                              max(peak, nbytes) / est)
                self.reserved += nbytes - resv
                self.resident[m] = Resident(m, handle, nbytes, False, t)
            else:
                results = out
                self.resident[m].busy = False
                self.resident[m].last_use = t
                self.resident.move_to_end(m)
            for r, z in zip(group, results):
                r.result, r.done, r.batch = z, t, len(group)
                done.append(r)
        self.inflight = keep
        return progressed

    @staticmethod
    def _cost(req):
        """Estimated device seconds of a request: a construction about half a
        microsecond per point (plus its product), a product on a resident
        matrix about a nanosecond per point and right-hand side."""
        n = req.rhs.shape[0]
        prod = 1e-9 * n * req.rhs.shape[1]
        return (5e-7 * n + prod) if req.points is not None else prod

    def _heavy(self, req):
        return req.points is not None and req.points.shape[0] >= self.heavy_points

    def _admit(self, pending, building, now, done):
        """One admission pass over the waiting requests: shortest estimated
        work first, less the time already waited times age_weight (so none
        starves), or in arrival order.  Products on resident matrices are
        admitted wherever they wait (they need no memory); constructions are
        considered among the first `lookahead` candidates only, and at most
        max_heavy constructions of heavy_points or more run at once (large
        builds that overlap slow each other and everything behind them)."""
        progressed = False
        scanned = 0
        t0 = now()
        if self.shortest_first:
            cands = sorted(pending, key=lambda r: self._cost(r)
                           - self.age_weight * max(0.0, t0 - r.arrival))
        else:
            cands = list(pending)
        heavy = sum(1 for f, kind, grp, _, _ in self.inflight
                    if kind == "build" and self._heavy(grp[0]))
        for req in cands:
            if len(self.inflight) >= self.slots:
                break
            if req not in pending:  # served by an earlier product group
                continue
            m = req.matrix
            if req.points is not None:
                if scanned >= self.lookahead:
                    continue
                scanned += 1
                if self._heavy(req) and heavy >= self.max_heavy:
                    continue
            if m in building:        # its matrix is being built: wait for it
                continue
            if m in self.resident:
                res = self.resident[m]
                if res.busy:
                    continue
                # merge every waiting product of this matrix (up to the
                # right-hand-side cap) into one launch
                group, cols = [], 0
                for r in list(pending):
                    if r.matrix == m and (not group or
                                          cols + r.rhs.shape[1] <= self.max_batch_rhs):
                        group.append(r)
                        cols += r.rhs.shape[1]
                for r in group:
                    pending.remove(r)
                t = now()
                for r in group:
                    r.admitted = t
                res.busy = True
                res.last_use = t
                self.resident.move_to_end(m)
                fut = self.ex.submit_product(res.handle, group)
                self.inflight.append((fut, "product", group, 0, m))
                self.log.append(("product", m, len(group)))
                progressed = True
                continue
            if req.points is None:
                if any(r.matrix == m and r.points is not None for r in pending):
                    continue      # its construction is still waiting
                src = self.sources.get(m)
                if src is None:
                    req.error, req.done = "matrix %s is not resident" % m, now()
                    pending.remove(req)
                    done.append(req)
                    progressed = True
                    continue
                # evicted earlier: built again from the points it was built
                # from, with this product as the construction's own product
                req.points, req.params = src
                self.log.append(("rebuild", m))
            asked = self._evaluated(req)  # the request itself may ask for that form
            need = self._need(req, evaluated=asked)
            evaluated = asked
            wanted = {r.matrix for r in pending if r.points is None}
            fits = need <= self.budget and (self.reserved + need <= self.budget or
                                            self._evict_for(need, wanted))
            if need > self.budget and self.allow_evaluated and not asked:
                # the stored form can never fit: the coupling blocks are
                # evaluated inside each product instead (slower products,
                # no stored blocks); a stored form that only has to wait for
                # memory waits
                need_e = self._need(req, evaluated=True)
                if need_e <= self.budget:
                    need, evaluated = need_e, True
                    fits = self.reserved + need <= self.budget or self._evict_for(need, wanted)
            if not fits:
                if need > self.budget:
                    req.error, req.done = "footprint above the memory budget", now()
                    pending.remove(req)
                    done.append(req)
                    progressed = True
                # else: does not fit yet; let smaller ones pass
                continue
            if evaluated and not asked:
                req.params = dict(req.params, coupling="evaluated")
                self.log.append(("evaluated", m))
            pending.remove(req)
            req.admitted = now()
            self.sources[m] = (req.points, req.params)
            self.reserved += need
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            building.add(m)
            fut = self.ex.submit_build(req)
            self.inflight.append((fut, "build", [req], need, m))
            self.log.append(("build", m))
            heavy += 1 if self._heavy(req) else 0
            progressed = True
        self.peak_inflight = max(self.peak_inflight, len(self.inflight))
        return progressed

    def close(self):
        for res in self.resident.values():
            self.ex.release(res.handle)
        self.resident.clear()
        self.reserved = 0


def latency_stats(done):
    lat = np.array([r.done - r.arrival for r in done if r.error is None])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "completed": int(lat.size),
            "failed": int(sum(r.error is not None for r in done))}


# ---------------------------------------------------------------- GPU executor
class GpuExecutor:
    """Runs builds and products through the C library on `slots` worker
    threads, each with its own HIP stream (default priority).  allocator
    "torch": every handle takes its device memory from torch's caching
    allocator (smash_options alloc/free hooks), so torch's accounting covers
    the resident matrices as well as the vectors.  memory_fraction: the
    share of the device torch's allocator may hold, freed blocks it keeps
    cached included (the engine's budget counts only what the handles and
    vectors use); the rest stays free for the runtime's own allocations,
    such as the scratch memory of kernels that spill registers."""

    def __init__(self, slots=4, prior_ratios=None, allocator=None, memory_fraction=None):
        import torch
        self.torch = torch
        if memory_fraction is not None:
            torch.cuda.set_per_process_memory_fraction(float(memory_fraction))
        self.pool = ThreadPoolExecutor(max_workers=slots)
        self.local = threading.local()
        self.prior = prior_ratios or {}
        self.allocator = allocator

    def _stream(self):
        s = getattr(self.local, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream()
            self.local.stream = s
        return s

    def estimate(self, req, evaluated=False):
        from . import api
        p = req.params
        n = max(req.rhs.shape[0], 1 if req.points is None else req.points.shape[0])
        dim = req.points.shape[1] if req.points is not None else p.get("dim", 2)
        return api.estimate_footprint(n, dim, p["kernel"], p["leaf"], p["order"], p["adm"],
                                      p["tol"], p["apply_prec"],
                                      coupling="evaluated" if evaluated else "stored")

    def prior_ratio(self, req):
        return self.prior.get(req.points.shape[1] if req.points is not None else 0, 1.0)

    def submit_build(self, req):
        return self.pool.submit(self._build, req)

    def submit_product(self, handle, group):
        return self.pool.submit(self._product, handle, group)

    def _build(self, req):
        from . import api
        torch = self.torch
        s = self._stream()
        p = dict(req.params)
        p.pop("dim", None)
        with torch.cuda.stream(s):
            X = torch.from_numpy(np.ascontiguousarray(req.points)).to("cuda", non_blocking=False)
            # graphs off: a graph replays only for a repeated argument set
            # (the same X and Y buffers), which fresh per-request vectors
            # never are
            try:
                h = api.Smash(X, stream=s, nrhs_hint=req.rhs.shape[1],
                              allocator=self.allocator, graphs=False, **p)
            except api.SmashError as e:
                if e.code == SMASH_E_OOM:
                    torch.cuda.empty_cache()  # cached blocks back before a retry
                raise
            dt = torch.float64 if h.apply_prec == "f64" else torch.float32
            Q = torch.from_numpy(np.ascontiguousarray(req.rhs)).to(dt).to("cuda")
            Z = h.matvec(Q, stream=s)
            s.synchronize()
            z = Z.cpu().numpy()
            inf = h.info()
        return h, inf["device_bytes"], [z], inf["build_peak_bytes"]

    def _product(self, h, group):
        torch = self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            dt = torch.float64 if h.apply_prec == "f64" else torch.float32
            Q = np.concatenate([r.rhs for r in group], axis=1)
            Qd = torch.from_numpy(np.ascontiguousarray(Q)).to(dt).to("cuda")
            Z = h.matvec(Qd, stream=s)
            s.synchronize()
            z = Z.cpu().numpy()
        out, c = [], 0
        for r in group:
            k = r.rhs.shape[1]
            out.append(z[:, c:c + k])
            c += k
        return out

    def release(self, handle):
        handle.close()

    def shutdown(self):
        self.pool.shutdown(wait=True)


# ---------------------------------------------------------------- traces
# Chebyshev points per axis by dimension: the orders whose products stay
# within 1e-6 of exact rows with FP64 apply (measured: 3D clustered 1/r at
# 2^20 points, 6 per axis: 3.7e-7; 5 per axis: 4.4e-6)
SERVE_ORDER = {2: 8, 3: 6}
SERVE_LEAF = {2: 64, 3: 128}


def make_trace(num, rate_hz, n_range=(10_000, 1_000_000), nrhs_range=(1, 32), seed=0,
               reuse=0.3, apply_prec="f32", tol=1e-6):
    """Poisson arrivals of construct-and-apply requests: N log-uniform in
    n_range, dimension 2 or 3, uniform or clustered points, kernel in
    {log r, 1/r, exp(-r)}, 1-32 right-hand sides; a fraction `reuse` of the
    requests are products on the matrix of an earlier request."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t = 0.0
    out, mats = [], []
    for rid in range(num):
        t += rng.exponential(1.0 / rate_hz)
        nr = int(rng.integers(nrhs_range[0], nrhs_range[1] + 1))
        if mats and rng.random() < reuse:
            m, n, params = mats[int(rng.integers(len(mats)))]
            rhs = rng.standard_normal((n, nr))
            out.append(Request(rid, t, m, rhs, None, dict(params)))
            continue
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        d = int(rng.choice([2, 3]))
        kind = "uniform" if rng.random() < 0.5 else "clusters"
        pts = W.uniform(n, d, 1000 + rid) if kind == "uniform" else W.clusters(n, d, 1000 + rid)
        kernel = ["log_r", "inv_r", "exp_r"][int(rng.integers(3))]
        params = dict(kernel=kernel, leaf=SERVE_LEAF[d], order=SERVE_ORDER[d], adm="strong",
                      tol=tol, apply_prec=apply_prec,
                      eval_prec="f64" if apply_prec == "f64" else "f32",
                      root=((0.0,) * d, 1.0), dim=d)
        m = "m%d" % rid
        mats.append((m, n, params))
        out.append(Request(rid, t, m, rng.standard_normal((n, nr)), pts, dict(params)))
    return out
