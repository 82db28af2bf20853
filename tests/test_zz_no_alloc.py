"""The entry point that allocates nothing (uhnsw_search_device_noalloc):
through the C-ABI, its results equal uhnsw_search_device's on the same
inputs, bit for bit, on two calls in a row (the second with fewer queries,
so stale contents of the shared fixed scratch region must not leak), in the
launch forms that use scratch; a search that needs more scratch than the
region, or asks for graph capture, is refused on the host before any
launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ctx_na(torch_cuda, wl1):
    from paper_2605_02030_amd import uhnsw

    wl, g1, g2 = wl1
    c = uhnsw.Context(0)
    c.load_graphs(wl.base, g1, g2)
    yield c
    c.close()


def _inputs(torch, wl, nq, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, wl.nq, nq)
    q = (wl.queries[idx] + rng.standard_normal((nq, wl.d)).astype(np.float32) * 0.05).astype(np.float32)
    p = (2.0 - 1.5 * rng.random(nq)).astype(np.float32)
    k = np.where(rng.random(nq) < 0.5, 10, 100).astype(np.int32)
    ef = rng.integers(k, 257).astype(np.int32)
    dev = torch.device("cuda:0")
    return tuple(torch.from_numpy(x).to(dev) for x in (q, p, k, ef))


def _run(torch, ctx, fn, inp, prm, with_stats, with_cand):
    from paper_2605_02030_amd import uhnsw

    q, p, k, ef = inp
    nq = q.shape[0]
    dev = torch.device("cuda:0")
    ids = torch.full((nq, 100), -7, dtype=torch.int64, device=dev)
    dists = torch.full((nq, 100), -7.0, dtype=torch.float32, device=dev)
    stats = torch.zeros((nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev) if with_stats else None
    cid = torch.empty((nq, 256), dtype=torch.int32, device=dev) if with_cand else None
    ckey = torch.empty((nq, 256), dtype=torch.float32, device=dev) if with_cand else None
    fn(q, p, k, ef, 100, 256, ids, dists, stats, cid, ckey, params=prm)
    torch.cuda.synchronize()
    out = [ids.cpu().numpy(), dists.cpu().numpy()]
    if with_stats:
        st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(nq)
        out += [st[f] for f in ("graph", "n_b", "n_exp", "n_p", "nc", "flags", "entry0", "n_up")]
    if with_cand:
        out += [cid.cpu().numpy(), ckey.cpu().numpy()]
    return out


FORMS = {"default": {}, "grid": dict(persistent=0), "counter": dict(persistent=1),
         "ordered-counter": dict(persistent=2), "fused": dict(fused=1),
         "fused-counter-beam2": dict(fused=1, persistent=1, beam_width=2)}


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("with_stats,with_cand", [(False, False), (True, False), (True, True)])
def test_noalloc_equals_search_device(torch_cuda, ctx_na, wl1, form, with_stats, with_cand):
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    prm = uhnsw.default_params(**FORMS[form])
    for call, nq in enumerate((300, 37)):  # the second call is smaller
        inp = _inputs(torch, wl, nq, seed=100 + call)
        want = _run(torch, ctx_na, ctx_na.search_device, inp, prm, with_stats, with_cand)
        got = _run(torch, ctx_na, ctx_na.search_device_noalloc, inp, prm, with_stats, with_cand)
        for a, b in zip(want, got):
            np.testing.assert_array_equal(a, b)
        if with_stats:
            assert (want[7] == 0).all()  # flags: every query searched


def test_noalloc_refusals(torch_cuda, ctx_na, wl1):
    """Refused on the host, before any launch: scratch above the fixed region
    (10,000 queries of the two-kernel form at ef_max 2048 need 164 MB of
    candidate lists), and graph capture or timing."""
    from paper_2605_02030_amd import uhnsw

    torch = torch_cuda
    wl, _, _ = wl1
    q, p, k, ef = _inputs(torch, wl, 10_000, seed=7)
    dev = torch.device("cuda:0")
    ids = torch.empty((10_000, 100), dtype=torch.int64, device=dev)
    dists = torch.empty((10_000, 100), dtype=torch.float32, device=dev)
    assert 10_000 * 2048 * 8 > uhnsw.UHNSW_NOALLOC_SCRATCH_BYTES
    with pytest.raises(uhnsw.UhnswError) as e:
        ctx_na.search_device_noalloc(q, p, k, ef, 100, 2048, ids, dists, params=uhnsw.default_params())
    assert e.value.code == uhnsw.UHNSW_EINVAL and "scratch" in str(e.value)
    for kw in (dict(graph=1), dict(timing=1)):
        with pytest.raises(uhnsw.UhnswError) as e:
            ctx_na.search_device_noalloc(q[:10], p[:10], k[:10], ef[:10], 100, 256, ids[:10], dists[:10],
                                         params=uhnsw.default_params(**kw))
        assert e.value.code == uhnsw.UHNSW_EINVAL
    # the same 10,000 queries fit in the fused form (no candidate lists), and
    # match the allocating entry point
    prm = uhnsw.default_params(fused=1)
    ids2 = torch.empty_like(ids)
    dists2 = torch.empty_like(dists)
    ctx_na.search_device(q, p, k, ef, 100, 256, ids, dists, params=prm)
    ctx_na.search_device_noalloc(q, p, k, ef, 100, 256, ids2, dists2, params=prm)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
    np.testing.assert_array_equal(dists.cpu().numpy(), dists2.cpu().numpy())
