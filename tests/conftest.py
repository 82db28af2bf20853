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
