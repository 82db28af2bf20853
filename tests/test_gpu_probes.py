"""GPU tests of the ceiling probes used to read the rooflines: they run,
return plausible rates, and reject row sizes the loaded rows cannot hold."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_probes(wl1):
    import torch

    from paper_2605_02030_amd import uhnsw

    assert torch.cuda.is_available()
    wl, g1, g2 = wl1
    ctx = uhnsw.Context(0)
    try:
        with pytest.raises(uhnsw.UhnswError):
            ctx.probe_gather(128)  # no index yet
        ctx.load_graphs(wl.base, g1, g2)  # d = 32: rows of 128 B
        gbs = ctx.probe_gather(128)
        assert math.isfinite(gbs) and gbs > 10.0
        for bad in (256, 512, 100):
            with pytest.raises(uhnsw.UhnswError):
                ctx.probe_gather(bad)
        ops = ctx.probe_transcendental()
        # 256 CUs x 16 lanes per cycle at most 2.4 GHz is about 9.8e12
        assert 1e11 < ops < 2e13
    finally:
        ctx.close()
