"""Pins for the oracle's walk under a fixed L_p (metric LP, the key
sum |x - q|^p of a graph built for one p: the per-p HNSW baseline of the
U-HNSW paper, Sec. 4.3) and for the per-p index variant.

Pins: p = 1 gives the L1 key bit for bit (each term |x - q| is exact); p =
0.5 on perfect-square differences gives the L0.5 key; on 0/1 coordinates
every term is 0 or 1 for any p, so the key counts the differing coordinates
exactly and a full-ef walk must return the brute-force Hamming top-t; on
real data the key stays within the FP32 summation bound of the FP64 sum;
a query whose p is the graph's stops after one verification batch."""
import numpy as np
import pytest

import oracle
import synth.graphs as sg
from test_oracle_search import _strongly_connected


def test_lp_key_p1_is_l1_bits():
    rng = np.random.Generator(np.random.PCG64(5))
    for g, v in ((8, 4), (16, 4), (4, 1)):
        for _ in range(20):
            x = rng.standard_normal(100).astype(np.float32)
            q = rng.standard_normal(100).astype(np.float32)
            assert oracle.base_dist(x, q, oracle.LP, g, v, mp=1.0) == oracle.base_dist(x, q, oracle.L1, g, v)


def test_lp_key_half_on_perfect_squares_is_l05(sq_workload):
    base, queries, _, _ = sq_workload
    for q in queries[:6]:
        for x in base[:50]:
            assert oracle.base_dist(x, q, oracle.LP, 8, 4, mp=0.5) == oracle.base_dist(x, q, oracle.L05, 8, 4)


@pytest.mark.parametrize("p", [0.3, 0.7, 1.2, 1.8])
def test_lp_key_counts_binary_differences(p):
    rng = np.random.Generator(np.random.PCG64(6))
    x = rng.integers(0, 2, size=(40, 64)).astype(np.float32)
    q = rng.integers(0, 2, size=64).astype(np.float32)
    for row in x:
        assert oracle.base_dist(row, q, oracle.LP, 8, 4, mp=p) == float((row != q).sum())


@pytest.mark.parametrize("p", [0.5, 0.7, 1.2, 1.8])
def test_lp_key_within_fp32_bound(p):
    rng = np.random.Generator(np.random.PCG64(7))
    d, g = 128, 8
    for _ in range(30):
        x = (rng.standard_normal(d) * 10).astype(np.float32)
        q = (rng.standard_normal(d) * 10).astype(np.float32)
        S64 = float((np.abs(x.astype(np.float64) - q.astype(np.float64)) ** p).sum())
        key = oracle.base_dist(x, q, oracle.LP, g, 4, mp=p)
        # each term rounded once (u), each lane sums d/g terms, log2(g) combines
        u = 2.0 ** -24
        bound = (1 + d // g + 3) * u * S64 * 1.01
        assert abs(key - S64) <= bound, (key, S64)


@pytest.fixture(scope="module")
def binary_workload():
    rng = np.random.Generator(np.random.PCG64(8))
    base = rng.integers(0, 2, size=(500, 16)).astype(np.float32)
    queries = rng.integers(0, 2, size=(8, 16)).astype(np.float32)
    g = sg.build_graph(base, sg.METRIC_L1, M=8, ef_construction=64, seed=3, cache=False)
    return base, queries, g


@pytest.mark.parametrize("p", [0.4, 1.3])
@pytest.mark.parametrize("w", [1, 2])
def test_full_ef_lp_walk_is_hamming_topt(binary_workload, p, w):
    base, queries, g = binary_workload
    assert _strongly_connected(g)
    G, D = oracle.Graph(g), oracle.Data(base)
    n = base.shape[0]
    for q in queries:
        ham = (base != q[None, :]).sum(1)
        order = np.lexsort((np.arange(n), ham))
        for t in (1, 10, 77, n):
            ids, keys, st = oracle.knn_search(G, D, q, oracle.LP, ef=n, t=t, w=w, mp=p)
            assert list(ids) == list(order[:t])
            np.testing.assert_array_equal(keys, ham[order[:t]].astype(np.float32))
            assert st.n_exp == n


def test_pgraph_same_p_stops_after_one_batch(wl1):
    """A query with the graph's own p: its walk keys and the verification's
    FP64 sums rank C alike unless two are within FP32 rounding, so almost
    every query stops after its first batch with R = C[0:K]."""
    wl, g1, _ = wl1
    p0 = 1.3
    gp = sg.build_graph(wl.base, sg.METRIC_L1, M=16, ef_construction=100, seed=4, cache=False)
    G = oracle.Graph(gp)
    prm = oracle.Params(variant=oracle.VARIANT_PGRAPH, walk_p=p0, cutoff=1e30)
    p = np.full(wl.nq, p0, np.float32)
    o = oracle.query_batch(G, G, oracle.Data(wl.base), wl.queries, p, wl.k, wl.ef, prm, c_stride=64)
    st = o["stats"]
    one = (st["batches"] == 1) & (st["n_p"] == np.minimum(st["nc"], wl.k + np.maximum(wl.k, 2)))
    assert one.mean() >= 0.95
    for i in np.flatnonzero(one):
        K = int(wl.k[i])
        assert set(o["ids"][i, :K].tolist()) == set(o["c_ids"][i, :K].tolist())
