"""Pins for the oracle's candidate verification (U-HNSW paper, Sec. 3.1 and
Algorithm 1) and the whole query path.

Pins: hand-traced runs of Algorithm 1 on one-dimensional data
(tests/golden/alg1_trace.json); tau > 1 with t = |C| = n equals the
brute-force L_p kNN (torch.cdist); the prefix invariant (the result is the
exact top-K of the first N_p candidates); p = 1 on G1 and p = 2 on G2 stop
after one batch with R = C[0:K] (the special case of Sec. 3); N_p is
monotone in tau; the partial-sum abort does not change results; m = ceil(tau K)
in exact decimal arithmetic.
"""
import fractions
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_m_of_exact_decimal():
    # 0.07, 0.14, 0.28, 0.55, 0.56 times 100 land just above an integer in binary
    for tau in ("0.92", "0.5", "0.9", "0.75", "0.95", "1.0", "0.1", "0.07", "0.14", "0.28", "0.55", "0.56"):
        for K in (1, 2, 3, 10, 25, 50, 100, 256):
            exact = math.ceil(fractions.Fraction(tau) * K)
            assert oracle.m_of(float(tau), K) == exact, (tau, K)
    assert [oracle.m_of(0.92, K) for K in (1, 10, 50, 100)] == [1, 10, 46, 92]


def test_alg1_hand_traces():
    with open(os.path.join(GOLD, "alg1_trace.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        x = np.array(c["x"], np.float32)
        if x.ndim == 1:
            x = x[:, None]
        D = oracle.Data(x)
        q = np.atleast_1d(np.array(c["q"], np.float32))
        C = np.array(c["C"], np.int32)
        m = oracle.m_of(c["tau"], c["K"])
        ids, S, dist, st = oracle.verify(D, q, c["p"], c["K"], C, c["kappa"], m, early_abort=c.get("abort", 1))
        assert list(ids) == c["ids"], c["name"]
        np.testing.assert_allclose(dist, c["dist"], rtol=1e-15)
        assert st.n_p == c["n_p"], c["name"]
        assert st.batches == c["batches"], c["name"]


@pytest.mark.parametrize("metric_graph", [1, 2])
def test_tau_above_one_is_bruteforce(small_int_workload, metric_graph):
    base, queries, g1, g2 = small_int_workload
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(base)
    n = base.shape[0]
    ps = np.array([0.5, 0.63, 0.9, 1.0, 1.2, 1.4, 1.41, 1.5, 1.77, 2.0] * 3, np.float32)[:len(queries)]
    prm = oracle.Params(tau=1.5, t_param=n)
    ef = np.full(len(queries), n, np.int32)
    k = np.full(len(queries), 10, np.int32)
    r = oracle.query_batch(G1, G2, D, queries, ps, k, ef, prm)
    for i in range(len(queries)):
        dd = torch.cdist(torch.from_numpy(queries[i:i + 1]).double(), torch.from_numpy(base).double(),
                         p=float(ps[i])).numpy()[0]
        order = np.lexsort((np.arange(n), dd))[:10]
        assert set(r["ids"][i]) == set(order)  # ties between equal distances may order by id only
        np.testing.assert_allclose(np.sort(r["dist"][i]), np.sort(dd[order]), rtol=1e-12)
        assert r["stats"]["n_p"][i] == n


def test_prefix_invariant_and_abort(wl1):
    wl, g1, g2 = wl1
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    a = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, oracle.Params(early_abort=1), c_stride=64)
    b = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, oracle.Params(early_abort=0), c_stride=64)
    np.testing.assert_array_equal(a["ids"], b["ids"])
    np.testing.assert_array_equal(a["dist"], b["dist"])
    np.testing.assert_array_equal(a["stats"]["n_p"], b["stats"]["n_p"])
    for i in range(wl.nq):
        npi = a["stats"]["n_p"][i]
        pref = a["c_ids"][i][:npi]
        dd = torch.cdist(torch.from_numpy(wl.queries[i:i + 1]).double(),
                         torch.from_numpy(wl.base[pref]).double(), p=float(wl.p[i])).numpy()[0]
        order = pref[np.lexsort((pref, dd))][:10]
        assert list(a["ids"][i]) == list(order)


def test_p1_p2_stop_after_first_batch(small_int_workload):
    """p = 1 uses G1 and p = 2 uses G2 (cutoff 1.4); on integer data the base key
    equals S_p exactly, so R = C[0:K] already holds the K best of the first batch."""
    base, queries, g1, g2 = small_int_workload
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(base)
    nq = len(queries)
    for p in (1.0, 2.0):
        ps = np.full(nq, p, np.float32)
        r = oracle.query_batch(G1, G2, D, queries, ps, np.full(nq, 10, np.int32), np.full(nq, 64, np.int32),
                               c_stride=64)
        st = r["stats"]
        assert (st["graph"] == (1 if p == 1.0 else 2)).all()
        assert (st["batches"] == 1).all() and (st["n_p"] == 20).all()
        np.testing.assert_array_equal(r["ids"][:, :10], r["c_ids"][:, :10])


def test_ext_stops_after_first_batch(sq_workload):
    """Extended variant (Sec. 4.5): p = 0.5 takes G_0.5 and p = 1 takes G_1
    (cutoff 0.6). With every |x - q| a perfect square, the L0.5 base key is
    the exact S_0.5 and the L1 key the exact S_1, so both stop after one
    batch with R = C[0:K], as p = 1, 2 do on the default pair."""
    base, queries, g05, g1 = sq_workload
    G05, G1, D = oracle.Graph(g05), oracle.Graph(g1), oracle.Data(base)
    nq = len(queries)
    prm = oracle.Params(variant=oracle.VARIANT_EXT, cutoff=0.6)
    for p, graph in ((0.5, 1), (1.0, 2)):
        ps = np.full(nq, p, np.float32)
        r = oracle.query_batch(G05, G1, D, queries, ps, np.full(nq, 10, np.int32), np.full(nq, 64, np.int32),
                               prm, c_stride=64)
        st = r["stats"]
        assert (st["graph"] == graph).all()
        assert (st["batches"] == 1).all() and (st["n_p"] == 20).all()
        np.testing.assert_array_equal(r["ids"][:, :10], r["c_ids"][:, :10])
        # and the result is the exact brute-force top-K (ties by id) where C reached it
        gt, _ = oracle.bruteforce(base, queries, ps, 10)
        assert np.mean(r["ids"][:, :10] == gt) > 0.9


def test_ext_graph_choice_cutoff(wl6):
    wl, g05, g1 = wl6
    G05, G1, D = oracle.Graph(g05), oracle.Graph(g1), oracle.Data(wl.base)
    ps = np.array([0.2, 0.5, np.float32(0.6), np.nextafter(np.float32(0.6), np.float32(1)), 0.8, 1.0], np.float32)
    n = len(ps)
    prm = oracle.Params(variant=oracle.VARIANT_EXT, cutoff=0.6)
    r = oracle.query_batch(G05, G1, D, wl.queries[:n], ps, np.full(n, 10, np.int32), np.full(n, 32, np.int32), prm)
    assert list(r["stats"]["graph"]) == [1, 1, 1, 2, 2, 2]


def test_ext_recall_and_bruteforce(wl6):
    """p over (0.2, 1] on the extended pair: recall@10 >= 0.9; with tau > 1
    and t = n every point is verified and the result is the brute force."""
    wl, g05, g1 = wl6
    G05, G1, D = oracle.Graph(g05), oracle.Graph(g1), oracle.Data(wl.base)
    prm = oracle.Params(variant=oracle.VARIANT_EXT, cutoff=0.6)
    r = oracle.query_batch(G05, G1, D, wl.queries, wl.p, wl.k, wl.ef, prm, c_stride=128)
    gt, _ = oracle.bruteforce(wl.base, wl.queries, wl.p, 10)
    rec = np.mean([len(set(r["ids"][i]) & set(gt[i])) / 10 for i in range(wl.nq)])
    rec0 = np.mean([len(set(r["c_ids"][i][:10]) & set(gt[i])) / 10 for i in range(wl.nq)])
    assert rec >= 0.9 and rec >= rec0
    n = 400
    sub = oracle.Data(wl.base[:n])
    import synth.graphs as sg

    h05 = sg.build_graph(wl.base[:n], sg.METRIC_L05, M=8, ef_construction=32, seed=3, cache=False)
    h1 = sg.build_graph(wl.base[:n], sg.METRIC_L1, M=8, ef_construction=32, seed=3, cache=False)
    nq = 12
    full = oracle.Params(variant=oracle.VARIANT_EXT, cutoff=0.6, tau=1.01, t_param=n)
    r = oracle.query_batch(oracle.Graph(h05), oracle.Graph(h1), sub, wl.queries[:nq], wl.p[:nq],
                           np.full(nq, 10, np.int32), np.full(nq, n, np.int32), full)
    assert (r["stats"]["nc"] == n).all()
    gt, _ = oracle.bruteforce(wl.base[:n], wl.queries[:nq], wl.p[:nq], 10)
    np.testing.assert_array_equal(r["ids"], gt)


def test_np_monotone_in_tau(wl1):
    wl, g1, g2 = wl1
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    prev = None
    for tau in (0.5, 0.7, 0.8, 0.92, 1.0, 1.01):
        r = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, oracle.Params(tau=tau))
        n_p = r["stats"]["n_p"]
        if prev is not None:
            assert (n_p >= prev).all()
        prev = n_p
    assert (prev == r["stats"]["nc"]).all()  # tau > 1: every candidate verified


def test_graph_choice_cutoff(wl1):
    wl, g1, g2 = wl1
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    ps = np.array([0.5, 1.0, np.float32(1.4), np.nextafter(np.float32(1.4), np.float32(2)), 1.5, 2.0], np.float32)
    n = len(ps)
    r = oracle.query_batch(G1, G2, D, wl.queries[:n], ps, np.full(n, 10, np.int32), np.full(n, 32, np.int32))
    assert list(r["stats"]["graph"]) == [1, 1, 1, 2, 2, 2]


def test_small_c_pads(small_int_workload):
    """|C| < K: the result has |C| entries; the rest of the row is -1 / +inf."""
    base, queries, g1, g2 = small_int_workload
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(base[:1])
    tiny1 = type(g1)(metric=1, n=1, M=8, ef_construction=64, seed=0, max_level=0, entry=0,
                     levels=np.zeros(1, np.int8),
                     layers=[type(g1.layers[0])(nodes=None, row_ptr=np.zeros(2, np.int64),
                                                col=np.zeros(0, np.int32))])
    T = oracle.Graph(tiny1)
    r = oracle.query_batch(T, T, D, queries[:2], np.array([0.7, 1.7], np.float32),
                           np.array([3, 3], np.int32), np.array([5, 5], np.int32))
    assert list(r["ids"][0]) == [0, -1, -1] and np.isinf(r["dist"][0][1:]).all()


def test_recall_cfg1(wl1):
    wl, g1, g2 = wl1
    G1, G2, D = oracle.Graph(g1), oracle.Graph(g2), oracle.Data(wl.base)
    r = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef)
    gt, _ = oracle.bruteforce(wl.base, wl.queries, wl.p, 10)
    rec = np.mean([len(set(r["ids"][i]) & set(gt[i])) / 10 for i in range(wl.nq)])
    assert rec >= 0.9
    # re-ranking never loses recall against the first K of C by base distance (Sec. 4.4, Table 2)
    r2 = oracle.query_batch(G1, G2, D, wl.queries, wl.p, wl.k, wl.ef, c_stride=64)
    rec0 = np.mean([len(set(r2["c_ids"][i][:10]) & set(gt[i])) / 10 for i in range(wl.nq)])
    assert rec >= rec0
