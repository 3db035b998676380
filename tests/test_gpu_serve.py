"""GPU test of the serving loop: requests served in a mix (overlapping on
the device through worker streams, products batched on resident matrices)
give the same results as each request served alone, within the FP32-apply
tolerance (1e-5 relative Frobenius)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1705_05443_amd import api, serve  # noqa: E402


@pytest.mark.parametrize("allocator", [None, "torch"])
def test_serving_mix_equals_alone(allocator):
    trace = serve.make_trace(12, rate_hz=400.0, n_range=(3000, 30000), nrhs_range=(1, 32),
                             seed=3, reuse=0.35)
    ex = serve.GpuExecutor(slots=4, allocator=allocator)
    eng = serve.Engine(ex, budget_bytes=64 << 30, slots=4)
    done = eng.run(trace)
    stats = serve.latency_stats(done)
    eng.close()
    ex.shutdown()
    print("serving", stats, "peak in flight", eng.peak_inflight, flush=True)
    assert len(done) == len(trace) and all(r.error is None for r in done), [r.error for r in done]
    assert eng.peak_inflight >= 2  # work of different requests overlapped
    points = {r.matrix: (r.points, r.params) for r in trace if r.points is not None}
    for r in sorted(done, key=lambda r: r.rid):
        pts, params = points[r.matrix]
        p = dict(params)
        p.pop("dim", None)
        h = api.Smash(torch.from_numpy(pts).cuda(), graphs=False, **p)
        z = h.matvec(torch.from_numpy(r.rhs.astype(np.float32)).cuda()).cpu().numpy()
        h.close()
        err = np.linalg.norm(r.result - z) / np.linalg.norm(z)
        assert err < 1e-5, (r.rid, r.matrix, err)


def test_serving_falls_back_to_evaluated_coupling():
    """A construction whose stored footprint exceeds the whole budget is
    served with its coupling blocks evaluated inside each product; its
    products equal those of the stored form built alone."""
    from paper_1705_05443_amd import workloads as W
    n, d = 30000, 2
    params = dict(kernel="log_r", leaf=serve.SERVE_LEAF[d], order=serve.SERVE_ORDER[d],
                  adm="strong", tol=1e-6, apply_prec="f32", eval_prec="f32",
                  root=((0.0,) * d, 1.0), dim=d)
    est = {c: api.estimate_footprint(n, d, params["kernel"], params["leaf"], params["order"],
                                     "strong", params["tol"], "f32", coupling=c)
           for c in ("stored", "evaluated")}
    budget = (est["stored"] + est["evaluated"]) // 2
    assert est["evaluated"] < budget < est["stored"], est
    rng = np.random.default_rng(11)
    pts = W.uniform(n, d, 77)
    reqs = [serve.Request(0, 0.0, "big", rng.standard_normal((n, 8)), pts, dict(params)),
            serve.Request(1, 0.001, "big", rng.standard_normal((n, 3)), None, dict(params))]
    ex = serve.GpuExecutor(slots=2)
    eng = serve.Engine(ex, budget_bytes=budget, slots=2)
    done = {r.rid: r for r in eng.run(reqs)}
    eng.close()
    ex.shutdown()
    assert all(r.error is None for r in done.values()), [r.error for r in done.values()]
    assert ("evaluated", "big") in eng.log
    p = dict(params)
    p.pop("dim")
    h = api.Smash(torch.from_numpy(pts).cuda(), graphs=False, coupling="stored", **p)
    for r in done.values():
        z = h.matvec(torch.from_numpy(r.rhs.astype(np.float32)).cuda()).cpu().numpy()
        err = np.linalg.norm(r.result - z) / np.linalg.norm(z)
        assert err < 1e-5, (r.rid, err)
    h.close()


def test_concurrent_constructions_match_one_stream():
    """Four constructions at once, each on a stream of its own (the register
    compr of every level is a grid of up to the device's resident workgroups
    whose groups wait for each other, so these launches are ordered across
    the streams), give the skeletons, ranks and product of the same
    construction made alone, bit for bit, over three rounds."""
    import threading

    from paper_1705_05443_amd import workloads as W
    kw = dict(kernel="inv_r", leaf=128, order=6, adm="strong", tol=1e-7, tau=0.7,
              root=((0.0, 0.0, 0.0), 1.0), graphs=False)
    sets = [W.clusters(12000 + 4000 * j, 3, seed=20 + j) for j in range(4)]
    qs = [W.rhs(x.shape[0], 4, seed=j) for j, x in enumerate(sets)]

    def one(j, stream):
        with torch.cuda.stream(stream):
            h = api.Smash(torch.from_numpy(sets[j]).cuda(), stream=stream, **kw)
            z = h.matvec(torch.from_numpy(qs[j]).cuda(), stream=stream)
            stream.synchronize()
            out = (h.export("ranks").copy(), h.export("row_sel").copy(), z.cpu().numpy())
            h.close()
        return out

    alone = [one(j, torch.cuda.current_stream()) for j in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    for rnd in range(3):
        got = [None] * 4
        errs = []
        start = threading.Barrier(4)

        def work(j):
            try:
                start.wait()
                got[j] = one(j, streams[j])
            except Exception as e:  # reported below
                errs.append((j, repr(e)))

        ts = [threading.Thread(target=work, args=(j,)) for j in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        print("round", rnd, "errors", errs, flush=True)
        assert not errs, errs
        for j in range(4):
            for a, b in zip(alone[j], got[j]):
                assert np.array_equal(a, b), (rnd, j)
