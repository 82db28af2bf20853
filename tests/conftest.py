import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def small_int_workload():
    """Tiny integer-valued data (exact FP32 base keys) with its two graphs."""
    import numpy as np
    import synth.graphs as sg

    rng = np.random.Generator(np.random.PCG64(7))
    base = rng.integers(0, 16, size=(600, 8)).astype(np.float32)
    queries = rng.integers(0, 16, size=(24, 8)).astype(np.float32)
    g1 = sg.build_graph(base, 1, M=8, ef_construction=64, seed=11, cache=False)
    g2 = sg.build_graph(base, 2, M=8, ef_construction=64, seed=11, cache=False)
    return base, queries, g1, g2


@pytest.fixture(scope="session")
def wl1():
    import synth
    import synth.graphs as sg

    wl = synth.make_workload(1)
    g1, g2 = sg.build_graphs(wl, cache=False)
    return wl, g1, g2


@pytest.fixture(scope="session")
def sq_workload():
    """Coordinates from {0, 16, 25}: every difference (16, 25, 9) is a
    perfect square, so L0.5 keys sum exact integer roots (3, 4, 5), and they
    rank differently from L1 keys (e.g. 3 + 3 > 5 but 9 + 9 < 25). Returns
    (base, queries, G_0.5, G_1), the extended variant's graph pair."""
    import numpy as np
    import synth.graphs as sg

    rng = np.random.Generator(np.random.PCG64(21))
    vals = np.array([0.0, 16.0, 25.0], np.float32)
    base = vals[rng.integers(0, 3, size=(600, 8))]
    queries = vals[rng.integers(0, 3, size=(24, 8))]
    g05 = sg.build_graph(base, sg.METRIC_L05, M=8, ef_construction=64, seed=11, cache=False)
    g1 = sg.build_graph(base, sg.METRIC_L1, M=8, ef_construction=64, seed=11, cache=False)
    return base, queries, g05, g1


@pytest.fixture(scope="session")
def wl6():
    """The extended variant's small workload: workload 1's vectors, p on
    (0.2, 1], graphs (G_0.5, G_1)."""
    import synth
    import synth.graphs as sg

    wl = synth.make_workload(6)
    g05, g1 = sg.build_graphs(wl, cache=False, extended=True)
    return wl, g05, g1
