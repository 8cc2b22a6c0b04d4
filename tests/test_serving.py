"""Serving loop: scheduling policy on the CPU; on the GPU, each request's result
is the same alone and in the continuous-batching mix (all three index kinds
resident at once, overlapping launches on several streams)."""
import numpy as np
import pytest

from paper_1509_03453_amd import serving as S
from paper_1509_03453_amd import workloads as W


# ---------------------------------------------------------------------------
# host-only policy
# ---------------------------------------------------------------------------
def test_pack_batch_takes_whole_requests_in_order():
    assert S.pack_batch([], 100) == 0
    assert S.pack_batch([10, 20, 30], 100) == 3
    assert S.pack_batch([10, 20, 30], 30) == 2
    assert S.pack_batch([10, 20, 30], 29) == 1
    assert S.pack_batch([500, 1], 100) == 1      # oversize head request goes alone
    assert S.pack_batch([50, 60, 10], 100) == 1  # no skipping ahead of a request that does not fit


def test_admissible_needs_reserve_and_cap():
    assert S.admissible(10, free_hbm=100, reserve=50, in_flight=0, pool_cap=20)
    assert not S.admissible(60, free_hbm=100, reserve=50, in_flight=0, pool_cap=1000)
    assert not S.admissible(10, free_hbm=100, reserve=50, in_flight=15, pool_cap=20)
    assert S.admissible(5, free_hbm=100, reserve=50, in_flight=15, pool_cap=20)


def test_latency_stats_percentiles():
    lat = np.arange(1, 101) * 1e-3  # 1..100 ms
    st = S.latency_stats(lat)
    assert st["p50_ms"] == pytest.approx(50.5)
    assert st["p99_ms"] == pytest.approx(99.01)
    assert st["max_ms"] == pytest.approx(100.0)
    assert S.latency_stats([])["p99_ms"] is None


def test_pick_index_is_first_come_first_served():
    import collections
    R = lambda t: S.Request(0, "x", np.zeros((1, 1)), t)  # noqa: E731
    qs = {"a": collections.deque([R(0.3)]), "b": collections.deque([R(0.1), R(0.5)]), "c": collections.deque()}
    assert S.pick_index(qs) == "b"
    assert S.pick_index({"a": collections.deque()}) is None


def test_graph_classes_pad_at_most_an_eighth():
    # one class per count the server can launch; a class covers every count
    # from the previous class + 1 up to itself, with at most 1/8 padding above 16
    c = S.graph_classes(8192)
    assert c[0] == 8 and c[1] == 16 and c[-1] == 8192
    assert all(a < b for a, b in zip(c, c[1:]))
    lo = 1
    for hi in c:
        for q in (lo, hi):
            assert q <= hi and (q <= 16 or 8 * (hi - q) < q), (q, hi)
        lo = hi + 1
    assert len(S.graph_classes(4096)) == 66 and S.graph_classes(10000)[-1] == 10240


def test_poisson_arrivals():
    reqs = W.serving_requests(20000, rate=500.0, n_indexes=3, max_q=4096)
    t = np.array([r[0] for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    assert gaps.mean() == pytest.approx(1 / 500.0, rel=0.03)
    assert gaps.std() == pytest.approx(1 / 500.0, rel=0.05)  # exponential: std == mean
    sizes = np.array([r[2] for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 4096
    assert sizes.mean() == pytest.approx(2048.5, rel=0.02)
    which = np.bincount([r[1] for r in reqs], minlength=3)
    assert which.min() > 0.3 * len(reqs)
    assert W.serving_requests(50, 10.0, 3) == W.serving_requests(50, 10.0, 3)


# ---------------------------------------------------------------------------
# GPU: invariance alone vs in the mix
# ---------------------------------------------------------------------------
def _make_mix(n_req, rate, max_q):
    import torch
    from paper_1509_03453_amd import binding as B
    from tests.gpu_util import dev, say

    say("[serving] building three resident indexes")
    g16 = W.gaussian_db(16384, 16, W.SEEDS["gauss16_db"])
    g64 = W.gaussian_db(60000, 64, W.SEEDS["gauss64_db"])
    d128 = W.descriptor_db(30000, 128)
    host = {"gauss16": (g16, 1), "gauss64": (g64, 2), "desc128": (d128, 2)}
    ixs = [S.ResidentIndex("gauss16", B.Index(dev(g16), 1, want_lowp=True), budget=512),
           S.ResidentIndex("gauss64", B.Index(dev(g64), 2, want_lowp=True), budget=2048),
           S.ResidentIndex("desc128", B.Index(dev(d128), 2, want_lowp=True), budget=1024)]

    def queries(name, n, seed):
        if name == "gauss16":
            return dev(W.gaussian_queries(n, 16, seed))
        if name == "gauss64":
            return dev(W.gaussian_queries(n, 64, seed))
        return dev(W.descriptor_queries(d128, n, pick_seed=seed, noise_seed=seed + 1)[0])

    names = [ix.name for ix in ixs]
    reqs = [S.Request(i, names[w], queries(names[w], n, s), a)
            for i, (a, w, n, s) in enumerate(W.serving_requests(n_req, rate, 3, max_q=max_q, seed=77))]
    torch.cuda.synchronize()
    return ixs, reqs, queries, host


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["tiled", "fp32"])
def test_serving_mix_equals_alone(orc, mode):
    import torch
    from paper_1509_03453_amd import binding as B
    from tests.gpu_util import candidates_of, check_screened, say

    ixs, reqs, queries, host = _make_mix(n_req=60, rate=3000.0, max_q=700)
    m = B.OS_ANN_MODE_TILED if mode == "tiled" else B.OS_ANN_MODE_FP32
    for ix in ixs:
        ix.mode = m
    srv = S.Server(ixs, slots=4, max_batch=1024, pool_cap_bytes=1 << 30, reserve_bytes=256 << 20)
    srv.warmup({ix.name: queries(ix.name, 1024, 99) for ix in ixs})
    say(f"[serving] mode={mode} running {len(reqs)} requests")
    st = srv.run(reqs, max_seconds=120)
    say(f"[serving] {st}")
    assert st["requests"] == len(reqs)
    assert st["queries"] == sum(r.n for r in reqs)
    assert st["batches"] < len(reqs)           # requests were packed together
    assert st["max_concurrent_launches"] >= 2  # launches overlapped on several streams
    assert st["p99_ms"] >= st["p50_ms"] > 0
    # the two clocks are tied to within tens of microseconds, steadily
    assert abs(st["clock_offset_us"]["drift"]) < 200 and st["clock_offset_us"]["before_spread"] < 500
    byname = {ix.name: ix for ix in ixs}
    for r in reqs:
        assert r.done is not None and r.latency > 0 and r.lag >= 0
        ix = byname[r.index]
        i1, d1, _ = B.os_ann_search_ex(ix.index.handle, r.queries, ix.budget, mode=m, rerank_r=ix.rerank_r)
        torch.cuda.synchronize()
        assert torch.equal(i1, r.out_idx), f"request {r.rid} ({r.index}, {r.n} queries): indices differ"
        assert torch.equal(d1, r.out_dist), f"request {r.rid}: distances differ"
    # what the server returned, against the oracle: every fifth request of each index
    oidx = {name: orc.build_index(X, L) for name, (X, L) in host.items()}
    for name, (X, L) in host.items():
        rr = [r for r in reqs if r.index == name][::5]
        Y = np.concatenate([r.queries.cpu().numpy() for r in rr])
        gi = torch.cat([r.out_idx for r in rr]).cpu().numpy()
        gd = torch.cat([r.out_dist for r in rr]).cpu().numpy()
        budget = byname[name].budget
        say(f"[serving] {mode} {name}: {len(rr)} served requests ({len(Y)} queries) against the oracle")
        if m == B.OS_ANN_MODE_FP32:
            oi, od32, od64, on = orc.search(X, oidx[name], Y, budget)
            assert np.array_equal(gi, oi), name
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), name
        else:
            o = orc.search_tiled(X, oidx[name], Y, budget, R=8)
            check_screened(orc, X, Y, (gi, gd, o[3]), o, ("serving", name),
                           is_candidate=candidates_of(orc, oidx[name], Y, budget))
    for ix in ixs:
        ix.index.close()


@pytest.mark.gpu
def test_serving_load_sweep():
    # saturation, then load points below it: every request is served, latency
    # parts are positive, and throughput does not exceed what was offered by
    # more than the arrival noise
    ixs, reqs, queries, host = _make_mix(n_req=8, rate=1.0, max_q=400)
    srv = S.Server(ixs, slots=4, max_batch=1024, pool_cap_bytes=1 << 30, reserve_bytes=256 << 20)
    srv.warmup({ix.name: queries(ix.name, 1024, 99) for ix in ixs})
    arrivals = W.serving_requests(260, 1.0, 3, max_q=400, seed=78)
    qs = [queries(ixs[w].name, n, sd) for (_, w, n, sd) in arrivals]

    def make(rate):
        t = [0.0 if rate == float("inf") else a / rate for (a, _, _, _) in arrivals]
        return [S.Request(i, ixs[w].name, qs[i], t[i]) for i, (_, w, _, _) in enumerate(arrivals)]

    out, last = S.load_sweep(srv, make, fractions=(0.5, 0.9), warmup_requests=20, saturation_requests=200)
    assert len(last) == 260 and all(r.out_idx is not None for r in last)
    assert out["saturation"]["req_per_s"] > 0
    for pt in out["points"]:
        assert pt["measured_requests"] == 240
        assert pt["p99_ms"] >= pt["p50_ms"] > 0
        assert pt["req_per_s"] <= 1.5 * pt["offered_req_per_s"]
    for ix in ixs:
        ix.index.close()


@pytest.mark.gpu
def test_serving_pool_cap_serialises_and_rejects():
    import torch
    from paper_1509_03453_amd import binding as B

    ixs, reqs, queries, host = _make_mix(n_req=12, rate=5000.0, max_q=300)
    need = max(S.Server(ixs).need_bytes(byn, 300, 128 * 4) for byn in ixs)
    srv = S.Server(ixs, slots=4, max_batch=300, pool_cap_bytes=need, reserve_bytes=0)
    st = srv.run(reqs, max_seconds=120)
    assert st["requests"] == len(reqs)
    assert srv.peak_in_flight <= need  # launches in flight never held more than the cap
    for r in reqs:
        ix = next(x for x in ixs if x.name == r.index)
        i1, d1, _ = B.os_ann_search_ex(ix.index.handle, r.queries, ix.budget, mode=ix.mode)
        torch.cuda.synchronize()
        assert torch.equal(i1, r.out_idx) and torch.equal(d1, r.out_dist)
    tiny = S.Server(ixs, slots=2, pool_cap_bytes=1024, reserve_bytes=0)
    with pytest.raises(MemoryError):
        tiny.run([S.Request(0, "gauss64", reqs[0].queries, 0.0)], max_seconds=30)
    for ix in ixs:
        ix.index.close()


@pytest.mark.gpu
def test_choose_mode_returns_the_faster_valid_mode():
    import torch
    from paper_1509_03453_amd import binding as B
    from tests.gpu_util import dev

    X = W.gaussian_db(50000, 64, seed=5101)
    Y = dev(W.gaussian_queries(2048, 64, seed=5102))
    ix = B.Index(dev(X), 2, want_lowp=True)
    try:
        for budget in (64, 20000):
            m = S.choose_mode(ix, Y, budget)
            assert m in (B.OS_ANN_MODE_FP32, B.OS_ANN_MODE_TILED)
            i, d, n = ix.search(Y, budget, mode=m)
            torch.cuda.synchronize()
            assert (i >= 0).all() and (i < 50000).all()
    finally:
        ix.close()
