"""GPU parity on the shapes of the five workloads.

* The benchmark workload (1M x 128 mixture, 10,000 queries) at full size in
  the launch configurations bench.py times, compared with the oracle on 527
  sampled queries; recall@10 against the stored FP64 ground truth.
* The precision form (d = 960 gamma features; BF16 and FP16 walk storage,
  FP32 re-rank), the batching form (d = 100 unit vectors, K in {1, 10,
  100}, ef in [K, 512]) and the serving form (d = 96 unit vectors, FP16 walk,
  K in {10, 100}) at reduced n with the full dimension.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import synth.graphs as sg  # noqa: E402
from test_gpu_parity import compare, run_device, _say  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def wl2_full():
    _say("workload 2 full size: generating inputs and graphs (cached when present)")
    wl = synth.make_workload(2)
    g1, g2 = sg.build_graphs(wl, cache=True, verbose=True)
    sys.stdout.flush()
    return wl, g1, g2


def _sample_compare(torch, ctx, wl, g1, g2, ef, params, storage, sample, w=1, variant=oracle.VARIANT_STD):
    """All queries on the GPU; the sample compared with the oracle."""
    from paper_2605_02030_amd import uhnsw

    g, v = ctx.layout()
    efa = np.full(wl.nq, ef, np.int32)
    ids, dists, st, cid, ckey = run_device(torch, ctx, wl.queries, wl.p, wl.k, efa, 10, ef, params=params)
    G1, G2 = oracle.Graph(g1), oracle.Graph(g2)
    D = oracle.Data(wl.base, storage=storage)
    sub = (ids[sample], dists[sample], st[sample], cid[sample], ckey[sample])
    compare(wl.base, G1, G2, D, wl.queries[sample], wl.p[sample], wl.k[sample], efa[sample], sub, g, v, w=w,
            variant=variant, cutoff=0.6 if variant == oracle.VARIANT_EXT else 1.4)
    assert (st["flags"] == 0).all()
    return ids


# 527 queries: the step 19 is prime to the 16-value p cycle, so every p of the
# grid is sampled about equally often
SAMPLE_STEP = 19


def bench_knobs(torch, ctx, wl, ef, uhnsw):
    """The batching form's knobs as bench.py picks them: autotuned fused
    launch (beam width, cache slots, waves per block, schedule, waves per CU)
    timed with two launches in flight, replayed as a hipGraph."""
    dev = torch.device("cuda:0")
    q = torch.from_numpy(wl.queries).to(dev)
    p = torch.from_numpy(wl.p).to(dev)
    k = torch.from_numpy(wl.k).to(dev)
    efa = torch.full((wl.nq,), ef, dtype=torch.int32, device=dev)
    base = uhnsw.default_params(fused=1, persistent=1, graph=1)
    t = ctx.autotune(q, p, k, efa, 10, ef, params=base, allow_beam=True, pipelined=True,
                     stream=torch.cuda.Stream())
    t.graph = 1
    return t


def _recall(ids, gt):
    got = ids[gt["qidx"], :10]
    return float(np.mean([len(set(got[i].tolist()) & set(gt["ids"][i].tolist())) / 10 for i in range(len(got))]))


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("form", ["fp32", "bf16-batched", "fp32-batched"])
def test_full_size_bench_configurations(torch_cuda, wl2_full, form):
    """The three forms bench.py times on the 1M x 128 workload at ef 256, in
    the launch configurations it times (the plain form at the default knobs;
    the batched forms autotuned and replayed from a captured hipGraph),
    against the oracle on 527 sampled queries covering all 16 p values, and
    recall@10 against the stored ground truth."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl2_full
    gt = dict(np.load(os.path.join(ROOT, "tests", "golden", "gt_mixture-1M-d128.npz")))
    assert bytes(gt["digest"]).decode() == wl.digest()
    sample = np.arange(3, wl.nq, SAMPLE_STEP)
    assert len(sample) >= 500 and len(set((sample % 16).tolist())) == 16
    ef = 256
    storage = uhnsw.STORE_BF16 if form == "bf16-batched" else uhnsw.STORE_F32
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(wl.base, g1, g2, storage=storage)
        prm = None if form == "fp32" else bench_knobs(torch_cuda, ctx, wl, ef, uhnsw)
        w = 1 if prm is None else prm.beam_width
        if prm is not None:
            _say(f"{form}: autotuned beam={prm.beam_width} slots={prm.visited_slots} wpb={prm.waves_per_block} "
                 f"persistent={prm.persistent} waves_per_cu={prm.waves_per_cu}")
        ids = _sample_compare(torch_cuda, ctx, wl, g1, g2, ef, prm, storage, sample, w=w)
    finally:
        ctx.close()
    rec = _recall(ids, gt)
    _say(f"full-size {form} recall@10 = {rec:.4f}")
    assert rec >= 0.9


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("slots,fused,beam", [(64, 0, 1), (128, 1, 2)])
def test_full_size_id_slot_cache(torch_cuda, wl2_full, slots, fused, beam):
    """Visited caches too small for 16-bit tags at a million ids: with 64
    slots a tag would need 20 - 6 + 3 = 17 bits, with 128 slots 16, so the
    cache holds 32-bit ids instead. A cache only decides which rows are
    gathered again, never which nodes enter W, so C and R still equal the
    oracle's (527 sampled queries; the walk gathers more rows)."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl2_full
    sample = np.arange(7, wl.nq, SAMPLE_STEP)
    prm = uhnsw.default_params(visited_slots=slots, fused=fused, beam_width=beam)
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(wl.base, g1, g2)
        _sample_compare(torch_cuda, ctx, wl, g1, g2, 128, prm, uhnsw.STORE_F32, sample, w=beam)
    finally:
        ctx.close()


@pytest.fixture(scope="module")
def wl7_full():
    _say("workload 7 full size (extended index): generating inputs and graphs (cached when present)")
    wl = synth.make_workload(7)
    g05, g1 = sg.build_graphs(wl, cache=True, verbose=True, extended=True)
    sys.stdout.flush()
    return wl, g05, g1


EF_EXT = 384  # bench.py --workload 7 calibrates to this efSearch (recall@10 0.928)


@pytest.mark.timeout(1200)
def test_full_size_extended(torch_cuda, wl7_full):
    """The extended index (G_0.5 + G_1, p over 0.2..1.0) on the benchmark's
    vectors in the launch configurations bench.py --workload 7 times."""
    from paper_2605_02030_amd import uhnsw

    wl, g05, g1 = wl7_full
    gt = dict(np.load(os.path.join(ROOT, "tests", "golden", f"gt_{wl.name}.npz")))
    assert bytes(gt["digest"]).decode() == wl.digest()
    sample = np.arange(5, wl.nq, SAMPLE_STEP)  # 527 queries, all 9 p values
    for storage, batched in ((uhnsw.STORE_F32, False), (uhnsw.STORE_BF16, True)):
        ctx = uhnsw.Context(0)
        ctx.load_graphs(wl.base, g05, g1, storage=storage, variant=uhnsw.VARIANT_EXT)
        prm = bench_knobs(torch_cuda, ctx, wl, EF_EXT, uhnsw) if batched else None
        ids = _sample_compare(torch_cuda, ctx, wl, g05, g1, EF_EXT, prm, storage, sample,
                              w=prm.beam_width if batched else 1, variant=oracle.VARIANT_EXT)
        ctx.close()
        got = ids[gt["qidx"], :10]
        rec = np.mean([len(set(got[i].tolist()) & set(gt["ids"][i].tolist())) / 10 for i in range(len(got))])
        _say(f"full-size extended storage={storage} recall@10 = {rec:.4f}")
        assert rec >= 0.9


@pytest.fixture(scope="module")
def wl3_small():
    wl = synth.make_workload(3, n=20_000, nq=48)
    g1, g2 = sg.build_graphs(wl, cache=False)
    return wl, g1, g2


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_precision_form_d960(torch_cuda, wl3_small, storage):
    """d = 960 rows (layout 64 lanes x 4 x 4 chunks, pitch 1024); BF16 / FP16
    walk with FP32 re-rank: C equals the oracle walking the same storage and
    distances stay within 1e-5 of FP64."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl3_small
    ctx = uhnsw.Context(0)
    ctx.load_graphs(wl.base, g1, g2, storage=storage)
    g, v = ctx.layout()
    assert (g, v) == (64, 4)
    efa = np.full(wl.nq, 128, np.int32)
    gpu = run_device(torch_cuda, ctx, wl.queries, wl.p, wl.k, efa, 10, 128)
    gpu_f = run_device(torch_cuda, ctx, wl.queries, wl.p, wl.k, efa, 10, 128,
                       params=uhnsw.default_params(fused=1, persistent=1))
    ctx.close()
    for a, b in zip(gpu[:2], gpu_f[:2]):
        np.testing.assert_array_equal(a, b)
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base, storage=storage)
    compare(wl.base, G1, G2, D, wl.queries, wl.p, wl.k, efa, gpu, g, v)


def test_partial_sum_abort_d960(torch_cuda):
    """The partial-sum abort on rows of 960 dimensions (half of each row
    summed; the other half read only while that partial sum is at most the
    K-th best S of R) changes no result. Input: tight clusters, with W (ef =
    t = 128) wider than a cluster, so C ends in members of other clusters;
    tau above 1 verifies all of C. Ids, distances, N_p and batches equal
    those with the abort off, in both kernel forms; with it on rows are
    really cut (n_cut > 0), with it off none are; the oracle agrees."""
    from paper_2605_02030_amd import uhnsw

    base, queries = synth.clustered(4000, 24, 960, clusters=80, seed=9301)
    nq = len(queries)
    p = np.array([0.5, 0.8, 1.0, 1.3, 1.6, 2.0], np.float32)[np.arange(nq) % 6]
    k = np.full(nq, 10, np.int32)
    efa = np.full(nq, 128, np.int32)
    g1 = sg.build_graph(base, sg.METRIC_L1, M=16, ef_construction=100, seed=7, cache=False)
    g2 = sg.build_graph(base, sg.METRIC_L2, M=16, ef_construction=100, seed=7, cache=False)
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(base, g1, g2)
        g, v = ctx.layout()
        assert g == 64
        for fused in (0, 1):
            prm = dict(fused=fused, t=128, tau=2.0)
            on = run_device(torch_cuda, ctx, queries, p, k, efa, 10, 128, params=uhnsw.default_params(**prm))
            off = run_device(torch_cuda, ctx, queries, p, k, efa, 10, 128,
                             params=uhnsw.default_params(early_abort=0, **prm))
            np.testing.assert_array_equal(on[0], off[0])
            np.testing.assert_array_equal(on[1], off[1])
            for f in ("n_p", "batches", "n_b", "n_exp"):
                np.testing.assert_array_equal(on[2][f], off[2][f])
            assert (off[2]["n_cut"] == 0).all()
            cut, n_p = int(on[2]["n_cut"].sum()), int(on[2]["n_p"].sum())
            _say(f"fused={fused}: abort cut {cut} of {n_p} L_p rows ({cut / n_p:.1%})")
            assert 0 < cut < n_p
    finally:
        ctx.close()
    compare(base, oracle.Graph(g1), oracle.Graph(g2), oracle.Data(base), queries, p, k, efa, on, g, v, tau=2.0,
            t_param=128)


@pytest.fixture(scope="module")
def wl4_small():
    wl = synth.make_workload(4, n=30_000, nq=300)
    g1, g2 = sg.build_graphs(wl, cache=False)
    return wl, g1, g2


def test_batching_form_d100_mixed(torch_cuda, wl4_small):
    """d = 100 (pitch padded to 128 with zeros), K in {1, 10, 100}, ef in
    [K, 512], one fused persistent launch against the oracle."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl4_small
    ctx = uhnsw.Context(0)
    ctx.load_graphs(wl.base, g1, g2)
    g, v = ctx.layout()
    gpu = run_device(torch_cuda, ctx, wl.queries, wl.p, wl.k, wl.ef, 100, 512,
                     params=uhnsw.default_params(fused=1, persistent=1))
    plain = run_device(torch_cuda, ctx, wl.queries, wl.p, wl.k, wl.ef, 100, 512)
    ctx.close()
    for a, b in zip(gpu[:2], plain[:2]):
        np.testing.assert_array_equal(a, b)
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    compare(wl.base, G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, gpu, g, v)


@pytest.fixture(scope="module")
def wl5_small():
    wl = synth.make_workload(5, n=30_000, nq=200)
    g1, g2 = sg.build_graphs(wl, cache=False)
    return wl, g1, g2


def test_serving_form_d96_fp16(torch_cuda, wl5_small):
    """The serving workload's shape at reduced n: d = 96 unit vectors (pitch
    padded to 128), FP16 walk with FP32 re-rank, K in {10, 100}, ef =
    max(K, 128). One fused launch and the same queries served as a Poisson
    mix at 100k/s: identical to each other, and C equal to the oracle walking
    the same FP16 storage, top-K by the near-tie rule."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl5_small
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(wl.base, g1, g2, storage=uhnsw.STORE_F16)
        g, v = ctx.layout()
        assert (g, v) == (8, 4)
        gpu = run_device(torch_cuda, ctx, wl.queries, wl.p, wl.k, wl.ef, 100, 128,
                         params=uhnsw.default_params(fused=1))
        srv = uhnsw.Server(ctx, k_max=100, ef_max=128)
        try:
            rng = np.random.Generator(np.random.PCG64(55))
            arrival = np.cumsum(rng.exponential(1e6 / 100_000, wl.nq))
            ids, dists, status, *_ = srv.drive(wl.queries, wl.p, wl.k, wl.ef, arrival)
        finally:
            srv.stop()
    finally:
        ctx.close()
    assert (status == 0).all()
    for i in range(wl.nq):
        K = int(wl.k[i])
        np.testing.assert_array_equal(ids[i, :K], gpu[0][i, :K])
        np.testing.assert_array_equal(dists[i, :K], gpu[1][i, :K])
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base, storage=oracle.F16)
    compare(wl.base, G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, gpu, g, v)


@pytest.mark.timeout(600)
def test_walk_reaches_half_hbm_peak(torch_cuda, wl2_full):
    """The plain FP32 walk on the benchmark workload (ef 256) moves at least
    half of MI355X's 8 TB/s in the method's own bytes: N_b rows of 512 B plus
    N_exp adjacency rows of 128 B per query, with N_b and N_exp from the
    oracle's walk over an exact visited set (rows the GPU's bounded visited
    cache forgot and gathered again are not counted), over the walk's own
    event time."""
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl2_full
    dev = torch_cuda.device("cuda:0")
    q = torch_cuda.from_numpy(wl.queries).to(dev)
    p = torch_cuda.from_numpy(wl.p).to(dev)
    k = torch_cuda.from_numpy(wl.k).to(dev)
    ef = torch_cuda.full((wl.nq,), 256, dtype=torch_cuda.int32, device=dev)
    ids = torch_cuda.empty((wl.nq, 10), dtype=torch_cuda.int64, device=dev)
    dists = torch_cuda.empty((wl.nq, 10), dtype=torch_cuda.float32, device=dev)
    stats = torch_cuda.zeros((wl.nq, uhnsw.STATS_WORDS), dtype=torch_cuda.int32, device=dev)
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(wl.base, g1, g2)
        g, v = ctx.layout()
        prm = uhnsw.default_params(timing=1)
        walk = []
        for _ in range(4):
            ctx.search_device(q, p, k, ef, 10, 256, ids, dists, stats, params=prm)
            walk.append(ctx.last_timing()[0])
        st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(wl.nq)
    finally:
        ctx.close()
    o = oracle.query_batch(oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base), wl.queries, wl.p, wl.k,
                           np.full(wl.nq, 256, np.int32), oracle.Params(g=g, v=v), threads=16)["stats"]
    np.testing.assert_array_equal(st["n_exp"], o["n_exp"])
    nbytes = float(o["n_b"].astype(np.float64).sum() * 512 + o["n_exp"].astype(np.float64).sum() * 128)
    gbs = nbytes / (min(walk[1:]) * 1e-3) / 1e9
    _say(f"walk {min(walk[1:]):.3f} ms, {gbs:,.0f} GB/s of the method's bytes; GPU rows / oracle rows "
         f"{st['n_b'].sum() / o['n_b'].sum():.3f}")
    assert gbs >= 0.5 * 8000.0
