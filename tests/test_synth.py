"""Seeded input generators and the HNSW base-graph builder (inputs to both
the oracle and the GPU path): determinism, shapes, value ranges, and the
structural invariants of an HNSW graph (Sec. 2.2 of the U-HNSW paper: a
layered proximity graph with at most M neighbours per node on upper layers
and 2M on layer 0)."""
import numpy as np
import pytest

import synth
import synth.graphs as sg


def test_workload_determinism_and_shapes():
    a = synth.make_workload(1)
    b = synth.make_workload(1)
    assert a.digest() == b.digest()
    assert a.base.shape == (10_000, 32) and a.queries.shape == (100, 32)
    assert a.base.dtype == np.float32 and (a.k == 10).all() and (a.ef == 64).all()
    assert ((a.p > 0.5) | (a.p == 0.5)).all() and (a.p <= 2.0).all()


def test_mixture_integer_range():
    w = synth.make_workload(2, n=5000, nq=64)
    assert w.base.shape == (5000, 128)
    assert (w.base == np.rint(w.base)).all() and w.base.min() >= 0 and w.base.max() <= 255
    np.testing.assert_array_equal(w.p[:16], synth.P_GRID)
    np.testing.assert_array_equal(w.p[16:32], synth.P_GRID)


def test_other_workloads_small():
    w3 = synth.make_workload(3, n=200, nq=5)
    assert (w3.base >= 0).all() and w3.d == 960
    w4 = synth.make_workload(4, n=300, nq=30)
    np.testing.assert_allclose(np.linalg.norm(w4.base, axis=1), 1.0, rtol=1e-5)
    assert list(w4.k[:6]) == [1, 10, 100, 1, 10, 100]
    assert (w4.ef >= w4.k).all() and (w4.ef <= 512).all()
    w5 = synth.make_workload(5, n=300, nq=50)
    assert set(np.unique(w5.k)) <= {10, 100} and w5.d == 96


@pytest.mark.parametrize("metric", [1, 2])
def test_graph_invariants(wl1, metric):
    wl, g1, g2 = wl1
    g = g1 if metric == 1 else g2
    n, M = g.n, g.M
    assert g.levels[g.entry] == g.max_level == g.levels.max()
    for l, L in enumerate(g.layers):
        nodes = np.arange(n) if l == 0 else L.nodes
        np.testing.assert_array_equal(nodes, np.nonzero(g.levels >= l)[0])
        deg = np.diff(L.row_ptr)
        assert deg.max() <= (2 * M if l == 0 else M)
        on_layer = np.zeros(n, bool)
        on_layer[nodes] = True
        assert on_layer[L.col].all()  # neighbours live on the same layer
        for r in range(0, len(nodes), max(1, len(nodes) // 200)):
            row = L.col[L.row_ptr[r]:L.row_ptr[r + 1]]
            assert nodes[r] not in row and len(set(row.tolist())) == len(row)
    assert np.diff(g.layers[0].row_ptr).min() >= 1


def test_level_law(wl1):
    wl, g1, _ = wl1
    frac = (g1.levels >= 1).mean()
    assert abs(frac - 1 / g1.M) < 0.02  # P(level >= 1) = exp(-1/mL) = 1/M


def test_builder_thread_independent():
    rng = np.random.Generator(np.random.PCG64(12))
    base = rng.standard_normal((3000, 16)).astype(np.float32)
    a = sg.build_graph(base, 2, M=8, ef_construction=40, seed=5, threads=1, cache=False)
    b = sg.build_graph(base, 2, M=8, ef_construction=40, seed=5, threads=7, cache=False)
    assert a.entry == b.entry and a.max_level == b.max_level
    for la, lb in zip(a.layers, b.layers):
        np.testing.assert_array_equal(la.row_ptr, lb.row_ptr)
        np.testing.assert_array_equal(la.col, lb.col)


def test_index_file_layouts(tmp_path):
    """The .fbin and UHG1 writers produce the documented layouts (read back
    here field by field; the C loader parses the same layout on the GPU)."""
    import synth
    import synth.graphs as sg

    wl = synth.make_workload(1, n=300, nq=4, d=8)
    g1, _ = sg.build_graphs(wl, cache=False)
    vp, gp = tmp_path / "v.fbin", tmp_path / "g1.uhg"
    sg.save_fbin(str(vp), wl.base)
    sg.save_graph_file(str(gp), g1)
    raw = vp.read_bytes()
    n, d = np.frombuffer(raw[:8], np.int32)
    assert (n, d) == (300, 8)
    np.testing.assert_array_equal(np.frombuffer(raw[8:], np.float32).reshape(n, d), wl.base)
    b = gp.read_bytes()
    assert b[:4] == b"UHG1"
    n2, M, ml, ep = np.frombuffer(b[4:20], np.int32)
    assert (n2, M, ml, ep) == (300, g1.M, g1.max_level, g1.entry)
    at = 20
    np.testing.assert_array_equal(np.frombuffer(b[at:at + n2], np.int8), g1.levels)
    at += n2
    for l, L in enumerate(g1.layers):
        nl = int(np.frombuffer(b[at:at + 8], np.int64)[0]); at += 8
        rp = np.frombuffer(b[at:at + 8 * (nl + 1)], np.int64); at += 8 * (nl + 1)
        np.testing.assert_array_equal(rp, L.row_ptr)
        col = np.frombuffer(b[at:at + 4 * rp[-1]], np.int32); at += 4 * int(rp[-1])
        np.testing.assert_array_equal(col, L.col)
        if l >= 1:
            nodes = np.frombuffer(b[at:at + 4 * nl], np.int32); at += 4 * nl
            np.testing.assert_array_equal(nodes, L.nodes)
    assert at == len(b)


def test_extended_workloads_share_vectors():
    """Workloads 6 and 7 (the extended variant's inputs) reuse workloads 1
    and 2's vectors, queries and graph seed; only p changes, to (0.2, 1]
    (6: uniform) and the 0.1 grid 0.2 .. 1.0 (7)."""
    a, b = synth.make_workload(1), synth.make_workload(6)
    assert np.array_equal(a.base, b.base) and np.array_equal(a.queries, b.queries)
    assert a.graph_seed == b.graph_seed
    assert (b.p > 0.2).all() and (b.p <= 1.0).all()
    c = synth.make_workload(7, n=2000)
    d = synth.make_workload(2, n=2000)
    assert np.array_equal(c.base, d.base) and np.array_equal(c.queries, d.queries)
    np.testing.assert_array_equal(np.unique(c.p), synth.P_GRID_EXT)


def test_builder_fixed_p_metric():
    """Metric 4 (sum |x - y|^p, a graph built for one p): at p = 1 every term
    is |x - y| exactly, so the graph equals the L1 graph edge for edge; at
    p = 0.7 it is a valid HNSW graph; p outside (0, 2] is refused."""
    rng = np.random.Generator(np.random.PCG64(31))
    base = rng.standard_normal((2000, 12)).astype(np.float32)
    a = sg.build_graph(base, sg.METRIC_L1, M=8, ef_construction=40, seed=3, cache=False)
    b = sg.build_graph(base, sg.METRIC_LP, M=8, ef_construction=40, seed=3, cache=False, metric_p=1.0)
    assert a.entry == b.entry and a.max_level == b.max_level
    for la, lb in zip(a.layers, b.layers):
        np.testing.assert_array_equal(la.row_ptr, lb.row_ptr)
        np.testing.assert_array_equal(la.col, lb.col)
    c = sg.build_graph(base, sg.METRIC_LP, M=8, ef_construction=40, seed=3, cache=False, metric_p=0.7)
    np.testing.assert_array_equal(c.levels, a.levels)  # the level draw does not depend on the metric
    assert any(not np.array_equal(x.col, y.col) for x, y in zip(a.layers, c.layers))
    for L in c.layers:
        assert np.diff(L.row_ptr).max() <= 16
    for bad in (0.0, -1.0, 2.5):
        with pytest.raises(ValueError):
            sg.build_graph(base, sg.METRIC_LP, M=8, ef_construction=40, seed=3, cache=False, metric_p=bad)
