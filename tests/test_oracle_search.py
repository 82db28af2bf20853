"""Pins for the oracle's candidate generation (HNSW KnnSearch, U-HNSW paper
Sec. 3.1 with HNSW's search as described in Sec. 2.2).

Pins: with ef = n on a strongly connected layer 0 every reachable node is
visited and never evicted, so C must equal the brute-force base-metric top-t
(integer data: FP32 keys are exact, the brute force is numpy int64);
any beam width w gives the same C there; a lossy visited cache gives the
same C as the exact visited set at any ef (result-exactness of the cache).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle


def _strongly_connected(g):
    L0 = g.layers[0]
    deg = np.diff(L0.row_ptr)
    rows = np.repeat(np.arange(g.n), deg)
    A = sp.csr_matrix((np.ones_like(rows), (rows, L0.col)), shape=(g.n, g.n))
    nc, _ = connected_components(A, directed=True, connection="strong")
    return nc == 1


def _int_key(base, q, metric):
    """Exact integer base keys. L0.5 (metric 3) needs every |x - q| to be a
    perfect square (the inputs of ``sq_workload``)."""
    dl = np.abs(base.astype(np.int64) - q.astype(np.int64)[None, :])
    if metric == 1:
        return dl.sum(1)
    if metric == 2:
        return (dl * dl).sum(1)
    r = np.rint(np.sqrt(dl)).astype(np.int64)
    assert (r * r == dl).all()
    return r.sum(1)


def _exact_base_topt(base, q, metric, t):
    key = _int_key(base, q, metric)
    order = np.lexsort((np.arange(base.shape[0]), key))
    return order[:t], key[order[:t]]


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("w", [1, 2, 4])
def test_full_ef_is_exact_topt(small_int_workload, metric, w):
    base, queries, g1, g2 = small_int_workload
    g = g1 if metric == 1 else g2
    assert _strongly_connected(g)
    G, D = oracle.Graph(g), oracle.Data(base)
    n = base.shape[0]
    for q in queries[:8]:
        for t in (1, 10, 57, n):
            ids, keys, st = oracle.knn_search(G, D, q, metric, ef=n, t=t, w=w)
            ref_ids, ref_keys = _exact_base_topt(base, q, metric, t)
            assert list(ids) == list(ref_ids)
            np.testing.assert_array_equal(keys, ref_keys.astype(np.float32))
            assert st.n_exp == n  # every node expanded exactly once


@pytest.mark.parametrize("w", [1, 2])
def test_full_ef_is_exact_topt_l05(sq_workload, w):
    base, queries, g, _ = sq_workload
    assert _strongly_connected(g)
    G, D = oracle.Graph(g), oracle.Data(base)
    n = base.shape[0]
    for q in queries[:8]:
        for t in (1, 10, 57, n):
            ids, keys, st = oracle.knn_search(G, D, q, oracle.L05, ef=n, t=t, w=w)
            ref_ids, ref_keys = _exact_base_topt(base, q, 3, t)
            assert list(ids) == list(ref_ids)
            np.testing.assert_array_equal(keys, ref_keys.astype(np.float32))
            assert st.n_exp == n


@pytest.mark.parametrize("slots", [16, 64, 256])
def test_lossy_cache_same_c(wl1, slots):
    wl, g1, g2 = wl1
    D = oracle.Data(wl.base)
    for metric, g in ((1, g1), (2, g2)):
        G = oracle.Graph(g)
        for qi in range(0, 100, 9):
            for ef in (16, 64, 128):
                a, ka, sa = oracle.knn_search(G, D, wl.queries[qi], metric, ef, ef)
                b, kb, sb = oracle.knn_search(G, D, wl.queries[qi], metric, ef, ef, cache_slots=slots)
                assert list(a) == list(b)
                np.testing.assert_array_equal(ka, kb)
                assert sb.n_b >= sa.n_b and sb.n_exp == sa.n_exp


def test_c_sorted_unique_and_keys_consistent(wl1):
    wl, g1, g2 = wl1
    D = oracle.Data(wl.base)
    G = oracle.Graph(g1)
    for qi in range(0, 100, 13):
        ids, keys, st = oracle.knn_search(G, D, wl.queries[qi], 1, 64, 64, g=8, v=4)
        assert len(set(ids.tolist())) == len(ids) == 64
        pairs = list(zip(keys.tolist(), ids.tolist()))
        assert pairs == sorted(pairs)
        for i, k in zip(ids[:5], keys[:5]):
            assert oracle.base_dist(wl.base[i], wl.queries[qi], 1, 8, 4) == k
        assert st.n_b >= 64 and st.n_exp >= 1


def test_ef_monotone_quality(wl1):
    """Larger ef only improves the best keys found (statistically: mean over queries)."""
    wl, g1, _ = wl1
    D, G = oracle.Data(wl.base), oracle.Graph(g1)
    k16 = np.mean([oracle.knn_search(G, D, q, 1, 16, 10)[1].mean() for q in wl.queries[:40]])
    k128 = np.mean([oracle.knn_search(G, D, q, 1, 128, 10)[1].mean() for q in wl.queries[:40]])
    assert k128 <= k16


def test_search_deterministic_threads(wl1):
    wl, g1, g2 = wl1
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    a = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, c_stride=64, threads=1)
    b = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, c_stride=64, threads=8)
    for key in ("ids", "c_ids"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["dist"], b["dist"])


def _textbook_search(g, base, q, metric, ef):
    """HNSW search as usually stated (HNSW paper's SEARCH-LAYER with a
    candidate min-heap and a result max-heap; greedy ef = 1 descent on the
    upper layers), keys (delta, id) with exact integer delta. Written with
    heaps, independently of the oracle's sorted-list formulation."""
    import heapq

    key = _int_key(base, q, metric)
    cur = g.entry
    for l in range(g.max_level, 0, -1):
        L = g.layers[l]
        changed = True
        while changed:
            changed = False
            r = int(np.searchsorted(L.nodes, cur))
            for e in L.col[L.row_ptr[r]:L.row_ptr[r + 1]]:
                if (key[e], e) < (key[cur], cur):
                    cur, changed = int(e), True
    start = cur
    L0 = g.layers[0]
    visited = {cur}
    C = [(key[cur], cur)]
    W = [(-key[cur], -cur)]
    while C:
        c = heapq.heappop(C)
        worst = (-W[0][0], -W[0][1])
        if c > worst:
            break
        for e in L0.col[L0.row_ptr[c[1]]:L0.row_ptr[c[1] + 1]]:
            e = int(e)
            if e in visited:
                continue
            visited.add(e)
            ke = (key[e], e)
            worst = (-W[0][0], -W[0][1])
            if len(W) < ef or ke < worst:
                heapq.heappush(C, ke)
                heapq.heappush(W, (-ke[0], -ke[1]))
                if len(W) > ef:
                    heapq.heappop(W)
    res = sorted((-a, -b) for a, b in W)
    return [i for _, i in res], start


@pytest.mark.parametrize("metric", [1, 2])
def test_matches_textbook_heap_search(small_int_workload, metric):
    base, queries, g1, g2 = small_int_workload
    g = g1 if metric == 1 else g2
    G, D = oracle.Graph(g), oracle.Data(base)
    for q in queries:
        for ef in (1, 3, 10, 32):
            ids, keys, st = oracle.knn_search(G, D, q, metric, ef=ef, t=ef)
            ref, start = _textbook_search(g, base, q, metric, ef)
            assert list(ids) == ref[:ef]
            assert st.entry0 == start


def test_matches_textbook_heap_search_l05(sq_workload):
    base, queries, g, _ = sq_workload
    G, D = oracle.Graph(g), oracle.Data(base)
    for q in queries:
        for ef in (1, 3, 10, 32):
            ids, keys, st = oracle.knn_search(G, D, q, oracle.L05, ef=ef, t=ef)
            ref, start = _textbook_search(g, base, q, 3, ef)
            assert list(ids) == ref[:ef]
            assert st.entry0 == start


def test_descent_ends_in_layer1_local_min(wl1):
    wl, g1, g2 = wl1
    D = oracle.Data(wl.base)
    for metric, g in ((1, g1), (2, g2)):
        assert g.max_level >= 1
        G = oracle.Graph(g)
        L = g.layers[1]
        moved = 0
        for q in wl.queries[:30]:
            _, _, st = oracle.knn_search(G, D, q, metric, 16, 16)
            e0 = st.entry0
            r = int(np.searchsorted(L.nodes, e0))
            assert L.nodes[r] == e0  # the descent ends on a layer-1 node
            k0 = oracle.base_dist(wl.base[e0], q, metric, 8, 4)
            for u in L.col[L.row_ptr[r]:L.row_ptr[r + 1]]:
                ku = oracle.base_dist(wl.base[u], q, metric, 8, 4)
                assert (ku, u) > (k0, e0)
            moved += e0 != g.entry
        assert moved > 0
