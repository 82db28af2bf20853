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
        # gfx950 issues v_exp_f32 / v_log_f32 at half the FP32 rate: 256 CUs x
        # 4 SIMDs x 16 lanes / 2 per cycle at 2.4 GHz = 19.66e12 lane-ops/s,
        # and the probe's chains put a full-rate multiply between the two
        # (at most 15.7e12); a quarter rate would cap it at 9.8e12
        assert 1e11 < ops <= 19.66e12 * 1.02
    finally:
        ctx.close()
