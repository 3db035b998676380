"""CPU tests of the serving scheduler with a host-only executor: admission
by footprint, slot limits, continuous admission, batching of products on a
resident matrix, eviction, and rejection of what can never fit."""
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from paper_1705_05443_amd.serve import Engine, Request, latency_stats


class FakeExecutor:
    """Builds take `build_s` seconds and hold real_per_point bytes per point
    (the estimate is 2 per point); products take `prod_s` seconds and
    return the right-hand sides times 2.  Tracks concurrency."""

    def __init__(self, slots, build_s=0.02, prod_s=0.005, real_per_point=1):
        self.pool = ThreadPoolExecutor(max_workers=slots)
        self.real = real_per_point
        self.build_s, self.prod_s = build_s, prod_s
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.released = []

    def estimate(self, req, evaluated=False):
        # the evaluated coupling form is estimated at a quarter of the stored one
        return (req.rhs.shape[0] // 2) if evaluated else 2 * req.rhs.shape[0]

    def prior_ratio(self, req):
        return 1.0

    def _enter(self):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)

    def _leave(self):
        with self.lock:
            self.running -= 1

    def _build(self, req):
        self._enter()
        time.sleep(self.build_s)
        self._leave()
        nb = self.real * req.rhs.shape[0]
        if req.params.get("coupling") == "evaluated":
            nb //= 4
        return ("H", req.matrix), nb, [2.0 * req.rhs]

    def _product(self, h, group):
        self._enter()
        time.sleep(self.prod_s)
        self._leave()
        return [2.0 * r.rhs for r in group]

    def submit_build(self, req):
        return self.pool.submit(self._build, req)

    def submit_product(self, h, group):
        return self.pool.submit(self._product, h, group)

    def release(self, h):
        self.released.append(h)


def _req(rid, t, m, n, nrhs=2, build=True):
    rhs = np.full((n, nrhs), float(rid))
    pts = np.zeros((n, 2)) if build else None
    return Request(rid, t, m, rhs, pts, {})


def test_all_requests_complete_within_slots_and_budget():
    ex = FakeExecutor(slots=3)
    eng = Engine(ex, budget_bytes=10_000, slots=3, margin=1.0)
    reqs = [_req(i, 0.002 * i, "m%d" % i, 1000 + 100 * i) for i in range(12)]
    done = eng.run(reqs)
    assert len(done) == 12 and all(r.error is None for r in done)
    assert ex.max_running <= 3 and eng.peak_inflight <= 3
    assert eng.peak_reserved <= 10_000
    for r in done:
        assert np.array_equal(r.result, 2.0 * r.rhs)
        assert r.admitted >= r.arrival and r.done >= r.admitted
    st = latency_stats(done)
    assert st["completed"] == 12 and st["p99_ms"] >= st["p50_ms"] > 0


def test_requests_admitted_while_others_run():
    """Continuous admission: a request arriving while earlier work is on the
    device starts before that work ends when a slot is free."""
    ex = FakeExecutor(slots=2, build_s=0.05)
    eng = Engine(ex, budget_bytes=10**9, slots=2)
    a, b = _req(0, 0.0, "a", 100), _req(1, 0.01, "b", 100)
    done = {r.rid: r for r in eng.run([a, b])}
    assert done[1].admitted < done[0].done


def test_products_on_a_resident_matrix_are_batched():
    ex = FakeExecutor(slots=1, build_s=0.03)
    eng = Engine(ex, budget_bytes=10**9, slots=1)
    reqs = [_req(0, 0.0, "m", 500)] + [_req(i, 0.001 * i, "m", 500, nrhs=3, build=False)
                                       for i in range(1, 6)]
    done = {r.rid: r for r in eng.run(reqs)}
    assert all(done[i].error is None for i in range(6))
    # five products waited for the build and went out as one launch
    assert [e for e in eng.log if e[0] == "product"] == [("product", "m", 5)]
    for i in range(1, 6):
        assert done[i].batch == 5 and np.array_equal(done[i].result, 2.0 * done[i].rhs)


def test_idle_residents_are_evicted_to_admit_new_builds():
    ex = FakeExecutor(slots=1, real_per_point=2)
    eng = Engine(ex, budget_bytes=3000, slots=1, margin=1.0, ratio=1.0, allow_evaluated=False)
    reqs = [_req(i, 0.0, "m%d" % i, 1000) for i in range(4)]  # 2000 reserved each
    done = eng.run(reqs)
    assert all(r.error is None for r in done)
    assert [e[1] for e in eng.log if e[0] == "evict"] == ["m0", "m1", "m2"]
    assert eng.peak_reserved <= 3000


def test_a_product_on_an_evicted_matrix_rebuilds_it():
    """A product that arrives after its matrix was evicted is served by
    building the matrix again from the points it was built from (the
    product rides on that construction), not failed."""
    ex = FakeExecutor(slots=1, real_per_point=2)
    eng = Engine(ex, budget_bytes=3000, slots=1, margin=1.0, ratio=1.0, allow_evaluated=False)
    reqs = [_req(i, 0.01 * i, "m%d" % i, 1000) for i in range(3)]  # m0, m1 evicted
    reqs.append(_req(9, 0.2, "m0", 1000, nrhs=3, build=False))
    done = {r.rid: r for r in eng.run(reqs)}
    assert all(r.error is None for r in done.values())
    assert ("rebuild", "m0") in eng.log
    assert np.array_equal(done[9].result, 2.0 * done[9].rhs)
    assert [e[1] for e in eng.log if e[0] == "build"] == ["m0", "m1", "m2", "m0"]


def test_a_request_that_can_never_fit_is_rejected():
    ex = FakeExecutor(slots=2)
    eng = Engine(ex, budget_bytes=1000, slots=2, ratio=1.0, margin=1.0)
    done = {r.rid: r for r in eng.run([_req(0, 0.0, "big", 5000), _req(1, 0.0, "ok", 100)])}
    assert done[0].error and "budget" in done[0].error
    assert done[1].error is None


def test_observed_bytes_calibrate_the_reservation():
    ex = FakeExecutor(slots=1)
    eng = Engine(ex, budget_bytes=10**9, slots=1, margin=1.0)
    eng.run([_req(0, 0.0, "a", 1000)])
    # real bytes are half the estimate: later reservations shrink to match
    assert abs(eng.ratios[(2, False)] - 0.5) < 1e-12
    assert eng._need(_req(1, 0.0, "b", 1000)) == 1000


def test_evaluated_coupling_admits_what_the_stored_form_cannot():
    """A construction whose stored footprint exceeds the budget is admitted
    with its coupling blocks evaluated inside each product (a quarter of the
    footprint here); without that fallback it is rejected."""
    ex = FakeExecutor(slots=1)
    eng = Engine(ex, budget_bytes=3000, slots=1, margin=1.0, ratio=1.0)
    done = {r.rid: r for r in eng.run([_req(0, 0.0, "big", 2000), _req(1, 0.01, "big", 2000,
                                                                        build=False)])}
    assert done[0].error is None and done[1].error is None
    assert ("evaluated", "big") in eng.log
    assert done[0].params.get("coupling") == "evaluated"
    assert np.array_equal(done[1].result, 2.0 * done[1].rhs)
    assert eng.peak_reserved <= 3000
    ex2 = FakeExecutor(slots=1)
    eng2 = Engine(ex2, budget_bytes=3000, slots=1, margin=1.0, ratio=1.0, allow_evaluated=False)
    d2 = eng2.run([_req(0, 0.0, "big", 2000)])
    assert d2[0].error and "budget" in d2[0].error


def test_a_request_for_the_evaluated_form_is_reserved_as_such():
    """A construction that asks for evaluated coupling blocks is reserved at
    the evaluated footprint (here a quarter of the stored one) from the start."""
    ex = FakeExecutor(slots=1)
    eng = Engine(ex, budget_bytes=1200, slots=1, margin=1.0, ratio=1.0, allow_evaluated=False)
    r = _req(0, 0.0, "e", 1000)
    r.params = dict(r.params, coupling="evaluated")
    done = eng.run([r])
    assert done[0].error is None
    assert eng.peak_reserved <= 1200


def test_waiting_product_keeps_its_matrix_resident():
    """A construction that needs memory must not evict a resident matrix that
    a waiting product request names (that request would fail as 'not
    resident'): the product is served first, then the matrix is evicted."""
    ex = FakeExecutor(slots=1, build_s=0.03, prod_s=0.01, real_per_point=2)
    eng = Engine(ex, budget_bytes=3000, slots=1, margin=1.0)
    reqs = [_req(0, 0.0, "m0", 1000),            # 2000 bytes: m0 and m1 do not fit together
            _req(1, 0.1, "m1", 1000),
            _req(2, 0.1, "m0", 1000, build=False)]
    done = eng.run(reqs)
    assert len(done) == 3 and all(r.error is None for r in done), [r.error for r in done]
    kinds = [e[:2] for e in eng.log]
    assert kinds.index(("product", "m0")) < kinds.index(("evict", "m0"))
    assert kinds.index(("evict", "m0")) < kinds.index(("build", "m1"))


def test_products_beyond_the_lookahead_are_admitted():
    """Products on resident matrices need no memory: they are admitted even
    when they wait behind more constructions than the lookahead considers."""
    ex = FakeExecutor(slots=2, build_s=0.02, prod_s=0.005)
    eng = Engine(ex, budget_bytes=2500, slots=2, margin=1.0, lookahead=2)
    reqs = [_req(0, 0.0, "m0", 1000)]
    reqs += [_req(1 + i, 0.05, "b%d" % i, 1200) for i in range(4)]
    reqs += [_req(9, 0.05, "m0", 1000, build=False)]
    done = eng.run(reqs)
    assert all(r.error is None for r in done), [r.error for r in done]
    r9 = [r for r in done if r.rid == 9][0]
    assert np.array_equal(r9.result, 2.0 * r9.rhs)


def test_shortest_first_admission():
    """With one slot and everything waiting at once, constructions run in
    order of estimated work (their point counts), not of arrival."""
    ex = FakeExecutor(slots=1, build_s=0.01)
    eng = Engine(ex, budget_bytes=10**9, slots=1, margin=1.0, age_weight=0.0)
    sizes = [5000, 1000, 3000, 2000, 4000]
    reqs = [_req(i, 0.0, "m%d" % i, n) for i, n in enumerate(sizes)]
    done = eng.run(reqs)
    order = [e[1] for e in eng.log if e[0] == "build"]
    assert order == ["m1", "m3", "m2", "m4", "m0"], order
    assert all(r.error is None for r in done)


def test_at_most_one_heavy_construction_in_flight():
    """Constructions of heavy_points or more points never overlap each other;
    smaller ones still run beside them."""
    class Ex(FakeExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.heavy_now = self.heavy_max = 0

        def _build(self, req):
            big = req.rhs.shape[0] >= 3000
            with self.lock:
                self.heavy_now += big
                self.heavy_max = max(self.heavy_max, self.heavy_now)
            out = super()._build(req)
            with self.lock:
                self.heavy_now -= big
            return out

    ex = Ex(slots=4, build_s=0.03)
    eng = Engine(ex, budget_bytes=10**9, slots=4, margin=1.0, heavy_points=3000)
    reqs = [_req(i, 0.0, "h%d" % i, 4000) for i in range(3)]
    reqs += [_req(10 + i, 0.0, "s%d" % i, 500) for i in range(3)]
    done = eng.run(reqs)
    assert len(done) == 6 and all(r.error is None for r in done)
    assert ex.heavy_max == 1
    assert ex.max_running >= 2  # small constructions overlapped the heavy ones


def test_constructions_reserve_their_peak_not_their_resident_size():
    """A construction's temporaries make its peak larger than what the
    finished matrix keeps: the engine learns that peak from the executor
    and reserves it while a construction runs, so resident matrices plus
    running constructions at their peak never exceed the budget."""
    class Ex(FakeExecutor):
        # estimate 2 per point; peak 1.5 per point; resident 0.5 per point
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.live = self.live_max = 0
            self.held = {}

        def _build(self, req):
            n = req.rhs.shape[0]
            with self.lock:
                self.live += 3 * n // 2
                self.live_max = max(self.live_max, self.live)
            self._enter()
            time.sleep(self.build_s)
            self._leave()
            with self.lock:
                self.live -= 3 * n // 2 - n // 2
                self.held[req.matrix] = n // 2
            return ("H", req.matrix), n // 2, [2.0 * req.rhs], 3 * n // 2

        def release(self, h):
            with self.lock:
                self.live -= self.held.pop(h[1])
            super().release(h)

    ex = Ex(slots=4, build_s=0.02)
    budget = 4000
    eng = Engine(ex, budget_bytes=budget, slots=4, margin=1.0, heavy_points=10**9)
    reqs = [_req(i, 0.001 * i, "m%d" % i, 1000) for i in range(16)]
    done = eng.run(reqs)
    assert len(done) == 16 and all(r.error is None for r in done)
    assert ex.live_max <= budget, ex.live_max
    assert eng.peak_ratios and max(eng.peak_ratios.values()) == 0.75


class _Oom(RuntimeError):
    code = -3  # SMASH_E_OOM


class OomOnceExecutor(FakeExecutor):
    """The first `fails` construction attempts of each matrix fail as the
    library does when an allocation fails (an error whose code is
    SMASH_E_OOM)."""

    def __init__(self, slots, fails=1, **kw):
        super().__init__(slots, **kw)
        self.fails = fails
        self.attempts = {}

    def _build(self, req):
        with self.lock:
            a = self.attempts.get(req.matrix, 0)
            self.attempts[req.matrix] = a + 1
        if a < self.fails:
            raise _Oom("allocator hook returned NULL")
        return super()._build(req)


def test_a_construction_that_runs_out_of_memory_is_queued_again():
    ex = OomOnceExecutor(slots=2, fails=1)
    eng = Engine(ex, budget_bytes=10**9, slots=2, margin=1.0)
    done = eng.run([_req(0, 0.0, "m0", 100), _req(1, 0.0, "m1", 120)])
    assert all(r.error is None for r in done) and len(done) == 2, [r.error for r in done]
    assert all(r.retries == 1 for r in done)
    assert ex.attempts == {"m0": 2, "m1": 2}
    assert sum(1 for e in eng.log if e[0] == "requeue") == 2
    assert eng.reserved == sum(r.bytes for r in eng.resident.values())
    eng.close()


def test_a_construction_that_keeps_running_out_of_memory_fails_after_the_retries():
    ex = OomOnceExecutor(slots=1, fails=10)
    eng = Engine(ex, budget_bytes=10**9, slots=1, margin=1.0, oom_retries=2)
    done = eng.run([_req(0, 0.0, "m0", 100)])
    assert len(done) == 1 and done[0].error is not None and done[0].retries == 2
    assert ex.attempts["m0"] == 3
    assert eng.reserved == 0
    eng.close()
