"""GPU test of loading the index from files (.fbin vectors, UHG1 graphs):
the searches equal those on the index loaded from memory, and damaged or
missing files are refused with UHNSW_EIO before anything is uploaded."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_load_graph_files(wl1, tmp_path):
    import torch

    import synth.graphs as sg
    from paper_2605_02030_amd import uhnsw

    assert torch.cuda.is_available()
    wl, g1, g2 = wl1
    vp, p1, p2 = (str(tmp_path / f) for f in ("base.fbin", "g1.uhg", "g2.uhg"))
    sg.save_fbin(vp, wl.base)
    sg.save_graph_file(p1, g1)
    sg.save_graph_file(p2, g2)
    a, b = uhnsw.Context(0), uhnsw.Context(0)
    try:
        a.load_graphs(wl.base, g1, g2)
        b.load_graph_files(vp, p1, p2)
        assert (b.n, b.d) == (wl.n, wl.d)
        ra = a.search(wl.queries, wl.p, wl.k, wl.ef, k_stride=10)
        rb = b.search(wl.queries, wl.p, wl.k, wl.ef, k_stride=10)
        np.testing.assert_array_equal(ra[0], rb[0])
        np.testing.assert_array_equal(ra[1], rb[1])
        # refused: missing file, truncated graph, graph of another size
        bad = str(tmp_path / "cut.uhg")
        with open(p1, "rb") as f, open(bad, "wb") as g:
            g.write(f.read()[:-7])
        for args in ((vp, p1, str(tmp_path / "none.uhg")), (vp, bad, p2)):
            with pytest.raises(uhnsw.UhnswError) as e:
                b.load_graph_files(*args)
            assert e.value.code == uhnsw.UHNSW_EIO
        small = str(tmp_path / "small.fbin")
        sg.save_fbin(small, wl.base[:100])
        with pytest.raises(uhnsw.UhnswError) as e:
            b.load_graph_files(small, p1, p2)
        assert e.value.code == uhnsw.UHNSW_EIO
    finally:
        a.close()
        b.close()
