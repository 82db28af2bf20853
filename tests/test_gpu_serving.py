"""GPU tests of the serving form (continuous batching): a query's result is
the same alone, in a Poisson mix, and in a plain batch search; admission
refuses work beyond its slots (EBUSY) and its HBM budget; batches that
arrive while others run overlap on the device."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from test_gpu_parity import _say  # noqa: E402


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ctxs(torch_cuda, wl1):
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    c = uhnsw.Context(0)
    c.load_graphs(wl.base, g1, g2)
    yield c
    c.close()


def _stream(wl, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, wl.nq, n)
    q = wl.queries[idx] + rng.standard_normal((n, wl.d)).astype(np.float32) * 0.05
    p = (2.0 - 1.5 * rng.random(n)).astype(np.float32)
    k = np.where(rng.random(n) < 0.5, 10, 100).astype(np.int32)
    ef = np.maximum(k, 128).astype(np.int32)
    return q.astype(np.float32), p, k, ef


def test_alone_vs_mix_vs_batch(torch_cuda, ctxs, wl1):
    from paper_2605_02030_amd import uhnsw

    wl, _, _ = wl1
    q, p, k, ef = _stream(wl, 3000, 41)
    srv = uhnsw.Server(ctxs, k_max=100, ef_max=128)
    try:
        # alone: one query at a time
        alone = {}
        for i in (0, 1, 777, 2999):
            assert srv.submit(q[i], p[i], k[i], ef[i], i) == uhnsw.UHNSW_OK
            got = []
            while not got:
                got = srv.poll()
            r = got[0]
            assert r.tag == i and r.status == 0
            alone[i] = (np.array(r.ids[:k[i]]), np.array(r.dists[:k[i]]))
        # in a mix: Poisson arrivals at 200k/s
        rng = np.random.Generator(np.random.PCG64(42))
        arrival = np.cumsum(rng.exponential(1e6 / 200_000, len(p)))
        ids, dists, status, t_sub, t_launch, t_done, st = srv.drive(q, p, k, ef, arrival, with_stats=True)
        info = srv.info()
    finally:
        srv.stop()
    _say("serving info", info)
    assert (status == 0).all()
    assert info["max_overlap"] >= 2  # batches overlapped on the device
    assert (t_done >= t_launch).all() and (t_launch >= t_sub - 1.0).all()
    for i, (ai, ad) in alone.items():
        np.testing.assert_array_equal(ids[i, :k[i]], ai)
        np.testing.assert_array_equal(dists[i, :k[i]], ad)
    # and equal to one plain batch launch of all queries
    ref_ids, ref_d, _ = ctxs.search(q, p, k, ef, params=uhnsw.default_params(fused=1), k_stride=100)
    for i in range(len(p)):
        np.testing.assert_array_equal(ids[i, :k[i]], ref_ids[i, :k[i]])
        np.testing.assert_array_equal(dists[i, :k[i]], ref_d[i, :k[i]])
    lat = t_done - t_sub
    _say(f"latency p50 {np.percentile(lat, 50):.0f} us p99 {np.percentile(lat, 99):.0f} us")
    # and against the oracle: the served rows and counters with C from a
    # device launch of the same queries (C is not part of a served result)
    import oracle
    from test_gpu_parity import compare, run_device

    _, g1, g2 = wl1
    g, v = ctxs.layout()
    _, _, _, cid, ckey = run_device(torch_cuda, ctxs, q, p, k, ef, 100, 128,
                                    params=uhnsw.default_params(fused=1))
    compare(wl.base, oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base), q, p, k, ef,
            (ids[:, :100], dists[:, :100], st, cid, ckey), g, v, label="served Poisson mix")


def test_admission_busy_and_budget(torch_cuda, ctxs, wl1):
    from paper_2605_02030_amd import uhnsw

    wl, _, _ = wl1
    q, p, k, ef = _stream(wl, 40, 43)
    srv = uhnsw.Server(ctxs, k_max=100, ef_max=128, max_inflight=4, streams=2)
    try:
        rcs = [srv.submit(q[i], p[i], k[i], ef[i], i) for i in range(40)]
        assert uhnsw.UHNSW_EBUSY in rcs
        accepted = [i for i, rc in enumerate(rcs) if rc == uhnsw.UHNSW_OK]
        assert 1 <= len(accepted) <= 40
        got = []
        while len(got) < len(accepted):
            got += srv.poll()
        assert sorted(r.tag for r in got) == accepted
        # slots are free again
        assert srv.submit(q[0], p[0], k[0], ef[0], 99) == uhnsw.UHNSW_OK
        while not srv.poll():
            pass
        assert srv.submit(q[0], 0.3, k[0], ef[0], 1) == uhnsw.UHNSW_EINVAL
        assert srv.submit(q[0], p[0], 101, 128, 1) == uhnsw.UHNSW_EINVAL
        # arrays the library would read past are refused by the binding
        with pytest.raises(ValueError):
            srv.submit(q[0][:-1], p[0], k[0], ef[0], 1)
        with pytest.raises(ValueError):
            srv.drive(q[:4], p[:3], k[:4], ef[:4], np.zeros(4))
        with pytest.raises(ValueError):
            srv.drive(q[:4], p[:4], k[:4], ef[:4], np.zeros(4), qidx=np.array([0, 1, 2, 4], np.int32))
    finally:
        srv.stop()
    with pytest.raises(uhnsw.UhnswError) as e:
        uhnsw.Server(ctxs, k_max=100, ef_max=128, hbm_budget=64)
    assert e.value.code == uhnsw.UHNSW_EBUSY


def test_admission_slots_follow_lds_plan(torch_cuda, ctxs):
    """Default slots = CUs x the fused kernel's resident waves per CU under
    the launch's LDS plan: a larger visited cache or list (more LDS per wave)
    admits fewer queries at once, never more."""
    from paper_2605_02030_amd import uhnsw

    waves = {}
    for slots, ef_max in ((1024, 128), (4096, 128), (8192, 128), (1024, 2048)):
        srv = uhnsw.Server(ctxs, k_max=100, ef_max=ef_max, params=uhnsw.default_params(visited_slots=slots))
        try:
            info = srv.info()
        finally:
            srv.stop()
        _say(f"visited slots {slots}, ef_max {ef_max}: {info['waves_per_cu']} waves per CU, "
             f"{info['slots']} query slots")
        assert info["slots"] == info["waves_per_cu"] * info["cus"]
        assert 1 <= info["waves_per_cu"] <= 32
        waves[(slots, ef_max)] = info["waves_per_cu"]
    assert waves[(1024, 128)] >= waves[(4096, 128)] >= waves[(8192, 128)]
    assert waves[(1024, 128)] > waves[(1024, 2048)]  # ef 2048: a 16 KiB list per wave


def test_reload_refused_while_serving(torch_cuda, wl1):
    """The server's thread searches on the context: replacing the index under
    it is refused until the server stops."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    c = uhnsw.Context(0)
    try:
        c.load_graphs(wl.base, g1, g2)
        srv = uhnsw.Server(c, k_max=10, ef_max=64)
        try:
            with pytest.raises(uhnsw.UhnswError) as e:
                c.load_graphs(wl.base, g1, g2)
            assert e.value.code == uhnsw.UHNSW_ESTATE
            assert srv.submit(wl.queries[0], float(wl.p[0]), 10, 64, 7) == uhnsw.UHNSW_OK
            got = []
            while not got:
                got = srv.poll()
            assert got[0].tag == 7 and got[0].status == 0
        finally:
            srv.stop()
        c.load_graphs(wl.base, g1, g2)  # allowed again
        ids, _, _ = c.search(wl.queries[:1], wl.p[:1], wl.k[:1], wl.ef[:1])
        assert (ids >= 0).all()
    finally:
        c.close()


def test_destroy_refused_while_serving(torch_cuda, wl1):
    """uhnsw_destroy leaves a context alone while a server runs on it;
    Context.close stops the servers first."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    c = uhnsw.Context(0)
    c.load_graphs(wl.base, g1, g2)
    srv = uhnsw.Server(c, k_max=10, ef_max=64)
    uhnsw.uhnsw_destroy(c.h)  # refused: the server's thread uses the context
    assert b"refused" in uhnsw.uhnsw_last_error(c.h)
    assert srv.submit(wl.queries[0], float(wl.p[0]), 10, 64, 3) == uhnsw.UHNSW_OK
    got = []
    while not got:
        got = srv.poll()
    assert got[0].tag == 3 and got[0].status == 0
    c.close()  # stops the server, then frees the context
    assert srv.h is None and c.h is None
