"""GPU construction of the HNSW base graphs (uhnsw_build_graph) against the
CPU input builder (synth/hnsw_build.c), which takes the same steps in the
same batch schedule with the same FP32 distance order: the two graphs must
be identical, level for level and edge for edge, for every base metric and
row layout, and at full size on the 1M x 128 benchmark vectors."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
import synth.graphs as sg  # noqa: E402
from test_gpu_parity import _say  # noqa: E402


@pytest.fixture(scope="module")
def ctx_b():
    import torch

    assert torch.cuda.is_available()
    from paper_2605_02030_amd import uhnsw

    c = uhnsw.Context(0)
    yield c
    c.close()


def assert_same_graph(a, b):
    assert a.M == b.M and a.max_level == b.max_level and a.entry == b.entry
    np.testing.assert_array_equal(np.asarray(a.levels), np.asarray(b.levels))
    assert len(a.layers) == len(b.layers)
    for l, (x, y) in enumerate(zip(a.layers, b.layers)):
        if l:
            np.testing.assert_array_equal(x.nodes, y.nodes)
        np.testing.assert_array_equal(x.row_ptr, y.row_ptr, err_msg=f"layer {l} row_ptr")
        np.testing.assert_array_equal(x.col, y.col, err_msg=f"layer {l} col")


CASES = [  # (workload, n, d, metric): row layouts of 1, 2 and 4 chunks of 64, d padded
    (1, 6000, 32, sg.METRIC_L1), (1, 6000, 32, sg.METRIC_L2), (1, 6000, 32, sg.METRIC_L05),
    (4, 5000, 100, sg.METRIC_L2), (2, 5000, 128, sg.METRIC_L1), (3, 3000, 200, sg.METRIC_L2),
]


@pytest.mark.parametrize("wl_id,n,d,metric", CASES)
def test_gpu_build_equals_cpu_builder(ctx_b, wl_id, n, d, metric):
    from paper_2605_02030_amd import uhnsw

    wl = synth.make_workload(wl_id, n=n, nq=1, d=d)
    base = wl.base
    for M, efc, bmax in ((16, 200, 1024), (8, 48, 16)):
        cpu = sg.build_graph(base, metric, M=M, ef_construction=efc, seed=11, cache=False, batch_max=bmax)
        gpu = uhnsw.build_graph(ctx_b, base, metric, M=M, ef_construction=efc, seed=11, batch_max=bmax)
        _say(f"build n={n} d={d} metric={metric} M={M} efc={efc} batch_max={bmax}: GPU {gpu.seconds:.2f}s "
             f"({gpu.batches} batches), max_level {gpu.max_level}, {len(gpu.layers[0].col)} layer-0 edges")
        assert_same_graph(cpu, gpu)


def test_gpu_build_refusals(ctx_b):
    from paper_2605_02030_amd import uhnsw

    base = np.zeros((10, 4), np.float32)
    for kw in (dict(metric=4), dict(M=1), dict(M=32), dict(ef_construction=0), dict(batch_max=0)):
        args = dict(metric=1, M=16, ef_construction=200, seed=0, batch_max=1024)
        args.update(kw)
        with pytest.raises(uhnsw.UhnswError) as e:
            uhnsw.build_graph(ctx_b, base, **args)
        assert e.value.code == uhnsw.UHNSW_EINVAL
    bad = base.copy()
    bad[3, 1] = np.inf
    with pytest.raises(uhnsw.UhnswError):
        uhnsw.build_graph(ctx_b, bad, 1)


@pytest.mark.timeout(900)
def test_gpu_build_full_size_equals_cached(ctx_b):
    """G1 and G2 of the 1M x 128 benchmark vectors built on the GPU equal the
    CPU builder's graphs (the cached ones every other test and bench.py use)."""
    from paper_2605_02030_amd import uhnsw

    wl = synth.make_workload(2)
    g1, g2 = sg.build_graphs(wl, cache=True, verbose=True)
    sys.stdout.flush()
    for metric, ref in ((sg.METRIC_L1, g1), (sg.METRIC_L2, g2)):
        gpu = uhnsw.build_graph(ctx_b, wl.base, metric, M=wl.M, ef_construction=wl.ef_construction,
                                seed=wl.graph_seed)
        _say(f"full-size build metric {metric}: {gpu.seconds:.1f}s on the GPU, {gpu.batches} batches")
        assert_same_graph(ref, gpu)
