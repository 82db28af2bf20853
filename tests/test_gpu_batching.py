"""GPU tests of the batching form: one fused walk+verify kernel, persistent
with a work counter over mixed p / k / ef, captured as a hipGraph, with
knobs chosen by the autotuner. Results must not depend on any of these."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from test_gpu_parity import compare, run_device, _say  # noqa: E402,F401


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ctxb(torch_cuda, wl1):
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    c = uhnsw.Context(0)
    c.load_graphs(wl.base, g1, g2)
    yield c
    c.close()


def _mixed(wl, seed=31):
    rng = np.random.Generator(np.random.PCG64(seed))
    nq = wl.nq
    k = np.array([1, 10, 100], np.int32)[np.arange(nq) % 3]
    ef = np.array([rng.integers(kk, 257) for kk in k], np.int32)
    p = wl.p.copy()
    p[:6] = [0.5, 1.0, 1.5, 2.0, 1.4, 0.73]
    return p, k, ef


def _same(a, b):
    for x, y in zip(a, b):
        if x.dtype.names:
            for f in x.dtype.names:
                if f not in ("n_b", "t_begin", "t_end"):
                    np.testing.assert_array_equal(x[f], y[f])
        else:
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("knobs", [dict(fused=1), dict(fused=1, persistent=0), dict(fused=1, persistent=1),
                                   dict(fused=1, persistent=2), dict(fused=1, persistent=3, beam_width=1),
                                   dict(fused=1, persistent=2, beam_width=1, visited_slots=1024),
                                   dict(fused=1, persistent=1, waves_per_cu=2),
                                   dict(fused=1, persistent=1, beam_width=1, visited_slots=256)])
def test_fused_matches_two_kernels(torch_cuda, ctxb, wl1, knobs):
    from paper_2605_02030_amd import uhnsw

    wl, _, _ = wl1
    p, k, ef = _mixed(wl)
    a = run_device(torch_cuda, ctxb, wl.queries, p, k, ef, 100, 256)
    b = run_device(torch_cuda, ctxb, wl.queries, p, k, ef, 100, 256, params=uhnsw.default_params(**knobs))
    _same(a, b)


def test_fused_persistent_parity_mixed(torch_cuda, ctxb, wl1):
    """Mixed p, K and ef in one persistent fused launch, against the oracle."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    g, v = ctxb.layout()
    p, k, ef = _mixed(wl, seed=32)
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    gpu = run_device(torch_cuda, ctxb, wl.queries, p, k, ef, 100, 256,
                     params=uhnsw.default_params(fused=1, persistent=1))
    compare(wl.base, G1, G2, D, wl.queries, p, k, ef, gpu, g, v)


def test_graph_replays(torch_cuda, ctxb, wl1):
    """Capture once, replay several times with eager work in between; every
    replay equals the eager result."""
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    dev = torch.device("cuda:0")
    p, k, ef = _mixed(wl, seed=33)
    nq = wl.nq
    tq = torch.from_numpy(wl.queries).to(dev)
    tp, tk, te = (torch.from_numpy(x).to(dev) for x in (p, k, ef))
    eager = run_device(torch, ctxb, wl.queries, p, k, ef, 100, 256, params=uhnsw.default_params(fused=1,
                                                                                                 persistent=1))
    ids = torch.empty((nq, 100), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, 100), dtype=torch.float32, device=dev)
    stats = torch.zeros((nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev)
    prm = uhnsw.default_params(fused=1, persistent=2, graph=1)  # cost-ordered: pre-pass kernels in the graph
    before = ctxb.graph_captures()
    for rep in range(4):
        ids.fill_(-7)
        dists.fill_(-7.0)
        ctxb.search_device(tq, tp, tk, te, 100, 256, ids, dists, stats, params=prm)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device=dev).sum()
        assert torch.isfinite(junk)
        np.testing.assert_array_equal(ids.cpu().numpy(), eager[0])
        np.testing.assert_array_equal(dists.cpu().numpy(), eager[1])
        st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(nq)
        np.testing.assert_array_equal(st["n_p"], eager[2]["n_p"])
    assert ctxb.graph_captures() == before + 1  # captured once, replayed after
    # changing an argument re-captures
    ctxb.search_device(tq, tp, tk, te, 100, 256, ids, dists, stats,
                       params=uhnsw.default_params(fused=1, persistent=1, graph=1, visited_slots=1024))
    torch.cuda.synchronize()
    assert ctxb.graph_captures() == before + 2
    np.testing.assert_array_equal(ids.cpu().numpy(), eager[0])


def test_autotune_result_invariant(torch_cuda, ctxb, wl1):
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    dev = torch.device("cuda:0")
    p, k, ef = _mixed(wl, seed=34)
    tq = torch.from_numpy(wl.queries).to(dev)
    tp, tk, te = (torch.from_numpy(x).to(dev) for x in (p, k, ef))
    tuned = ctxb.autotune(tq, tp, tk, te, 100, 256, params=uhnsw.default_params(fused=1))
    _say("autotuned", tuned.visited_slots, tuned.waves_per_block, tuned.persistent, tuned.beam_width)
    assert tuned.beam_width == 1 and tuned.fused == 1 and tuned.visited_slots in (1024, 2048, 4096)
    a = run_device(torch, ctxb, wl.queries, p, k, ef, 100, 256)
    b = run_device(torch, ctxb, wl.queries, p, k, ef, 100, 256, params=tuned)
    _same(a, b)
    again = ctxb.autotune(tq, tp, tk, te, 100, 256, params=uhnsw.default_params(fused=1))
    assert (again.visited_slots, again.waves_per_block, again.persistent) == \
        (tuned.visited_slots, tuned.waves_per_block, tuned.persistent)  # cached
    # timed as two launches in flight on two streams: knobs may differ, results may not
    piped = ctxb.autotune(tq, tp, tk, te, 100, 256, params=uhnsw.default_params(fused=1), pipelined=True,
                          stream=torch.cuda.Stream())
    _say("autotuned (pipelined)", piped.visited_slots, piped.waves_per_block, piped.persistent, piped.beam_width)
    assert piped.beam_width == 1 and piped.fused == 1
    c = run_device(torch, ctxb, wl.queries, p, k, ef, 100, 256, params=piped)
    _same(a, c)


def test_host_path_graph_with_copies(torch_cuda, ctxb, wl1):
    """Host-pointer search under a hipGraph: copies in, kernels, copies out are
    captured once per shape and replayed; each call's results equal the
    uncaptured search of the same queries."""
    from paper_2605_02030_amd import uhnsw

    wl, _, _ = wl1
    p, k, ef = _mixed(wl, seed=35)
    prm_g = uhnsw.default_params(fused=1, persistent=1, graph=1)
    prm_e = uhnsw.default_params(fused=1, persistent=1)
    before = ctxb.graph_captures()
    halves = (slice(0, 50), slice(50, 100))
    for rep in range(2):
        for sl in halves:  # same shape, different inputs: replay
            a = ctxb.search(wl.queries[sl], p[sl], k[sl], ef[sl], params=prm_g, k_stride=100)
            b = ctxb.search(wl.queries[sl], p[sl], k[sl], ef[sl], params=prm_e, k_stride=100)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
            np.testing.assert_array_equal(a[2]["n_p"], b[2]["n_p"])
    assert ctxb.graph_captures() == before + 1
    c = ctxb.search(wl.queries[:37], p[:37], k[:37], ef[:37], params=prm_g, k_stride=100)  # new shape
    d = ctxb.search(wl.queries[:37], p[:37], k[:37], ef[:37], params=prm_e, k_stride=100)
    np.testing.assert_array_equal(c[0], d[0])
    assert ctxb.graph_captures() == before + 2


def test_concurrent_streams(torch_cuda, ctxb, wl1):
    """Searches on two streams of one context at the same time (persistent,
    hipGraph-replayed, each stream with its own scratch) equal the same
    searches run one after another."""
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    dev = torch.device("cuda:0")
    p, k, ef = _mixed(wl, seed=36)
    tq = torch.from_numpy(wl.queries).to(dev)
    tp, tk, te = (torch.from_numpy(x).to(dev) for x in (p, k, ef))
    halves = (slice(0, 50), slice(50, 100))
    prm = uhnsw.default_params(fused=1, persistent=1, graph=1)
    ref = [run_device(torch, ctxb, wl.queries[h], p[h], k[h], ef[h], 100, 256, params=prm) for h in halves]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [(torch.full((50, 100), -7, dtype=torch.int64, device=dev),
             torch.full((50, 100), -7.0, dtype=torch.float32, device=dev),
             torch.zeros((50, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev)) for _ in halves]
    torch.cuda.synchronize()
    for rep in range(3):
        for h, st, (ids, dists, stats) in zip(halves, streams, outs):
            ctxb.search_device(tq[h], tp[h], tk[h], te[h], 100, 256, ids, dists, stats, params=prm, stream=st)
        torch.cuda.synchronize()
        for r, (ids, dists, stats) in zip(ref, outs):
            np.testing.assert_array_equal(ids.cpu().numpy(), r[0])
            np.testing.assert_array_equal(dists.cpu().numpy(), r[1])
            st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(50)
            np.testing.assert_array_equal(st["n_p"], r[2]["n_p"])
            np.testing.assert_array_equal(st["n_exp"], r[2]["n_exp"])


def test_graph_recaptured_after_scratch_grows(torch_cuda, ctxb, wl1):
    """A captured launch bakes in the per-stream scratch addresses (default
    stats, the cost-ordering pre-pass arrays). An uncaptured search of more
    queries on the same stream reallocates that scratch; the next captured
    search with the first call's arguments must capture again rather than
    replay into freed memory, and give the same results."""
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    dev = torch.device("cuda:0")
    p, k, ef = _mixed(wl, seed=37)
    tq = torch.from_numpy(wl.queries).to(dev)
    tp, tk, te = (torch.from_numpy(x).to(dev) for x in (p, k, ef))
    half = 50
    ids = torch.empty((half, 100), dtype=torch.int64, device=dev)
    dists = torch.empty((half, 100), dtype=torch.float32, device=dev)
    big_ids = torch.empty((wl.nq, 100), dtype=torch.int64, device=dev)
    big_dists = torch.empty((wl.nq, 100), dtype=torch.float32, device=dev)
    prm_g = uhnsw.default_params(fused=1, persistent=2, graph=1)  # stats left to the library's scratch
    prm_e = uhnsw.default_params(fused=1, persistent=2)
    ref = run_device(torch, ctxb, wl.queries[:half], p[:half], k[:half], ef[:half], 100, 256, params=prm_e)
    before = ctxb.graph_captures()
    ctxb.search_device(tq[:half], tp[:half], tk[:half], te[:half], 100, 256, ids, dists, params=prm_g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), ref[0])
    assert ctxb.graph_captures() == before + 1
    # a bigger uncaptured search on the same stream grows (moves) the scratch
    ctxb.search_device(tq, tp, tk, te, 100, 256, big_ids, big_dists, params=prm_e)
    torch.cuda.synchronize()
    for rep in range(2):
        ids.fill_(-7)
        ctxb.search_device(tq[:half], tp[:half], tk[:half], te[:half], 100, 256, ids, dists, params=prm_g)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ids.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(dists.cpu().numpy(), ref[1])
    assert ctxb.graph_captures() == before + 2  # captured again once, then replayed
