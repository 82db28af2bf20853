"""Recovery of a failed context (uhnsw_reset). The failure is forced from the
host: a search whose candidate-list scratch (nq x ef_max x 4 bytes, 17.6 TB
here) cannot be allocated fails with ENOMEM before any kernel is launched,
and marks the context failed."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from test_gpu_parity import _say, run_device  # noqa: E402


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available()
    return torch


def test_reset_after_failed_allocation(torch_cuda, wl1):
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, g1, g2 = wl1
    dev = torch.device("cuda:0")
    ctx = uhnsw.Context(0)
    try:
        ctx.load_graphs(wl.base, g1, g2)
        efa = np.full(wl.nq, 64, np.int32)
        ref = run_device(torch, ctx, wl.queries, wl.p, wl.k, efa, 10, 64)
        tq = torch.from_numpy(wl.queries).to(dev)
        tp = torch.from_numpy(wl.p).to(dev)
        tk = torch.from_numpy(wl.k).to(dev)
        te = torch.from_numpy(efa).to(dev)
        ids = torch.empty((wl.nq, 10), dtype=torch.int64, device=dev)
        dists = torch.empty((wl.nq, 10), dtype=torch.float32, device=dev)
        stats = torch.zeros((wl.nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev)
        huge = 2**31 - 1  # rows the host sizes scratch for; no kernel runs: the allocation fails first
        assert huge * uhnsw.UHNSW_EFMAX * 4 > 10 * 288e9
        stream = torch.cuda.current_stream().cuda_stream
        rc = uhnsw.uhnsw_search_device(ctx.h, tq.data_ptr(), huge, tp.data_ptr(), tk.data_ptr(), te.data_ptr(), 10,
                                       uhnsw.UHNSW_EFMAX, None, 10, ids.data_ptr(), dists.data_ptr(),
                                       stats.data_ptr(), None, None, 0, stream)
        msg = uhnsw.uhnsw_last_error(ctx.h).decode()
        _say("forced failure:", rc, msg)
        assert rc in (uhnsw.UHNSW_ENOMEM, uhnsw.UHNSW_EDEVICE), (rc, msg)
        # the failed context refuses work until reset
        rc = uhnsw.uhnsw_search_device(ctx.h, tq.data_ptr(), wl.nq, tp.data_ptr(), tk.data_ptr(), te.data_ptr(),
                                       10, 64, None, 10, ids.data_ptr(), dists.data_ptr(), stats.data_ptr(), None,
                                       None, 0, stream)
        assert rc == uhnsw.UHNSW_ESTATE, uhnsw.uhnsw_last_error(ctx.h).decode()
        ctx.reset()
        again = run_device(torch, ctx, wl.queries, wl.p, wl.k, efa, 10, 64)
        for a, b in zip(ref[:2], again[:2]):
            np.testing.assert_array_equal(a, b)
        ctx.reset()  # a healthy context resets the same way
        np.testing.assert_array_equal(run_device(torch, ctx, wl.queries, wl.p, wl.k, efa, 10, 64)[0], ref[0])
    finally:
        ctx.close()
