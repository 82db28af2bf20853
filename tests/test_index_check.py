"""Host-side index validation through the C-ABI, with no device: the checks
uhnsw_load_graphs makes before any upload (a graph that passed them is what
the kernels index without bounds checks), and the file form's refusals.
Each case damages one field of a valid index built by the HNSW builder."""
import copy

import numpy as np
import pytest

import synth
import synth.graphs as sg


@pytest.fixture(scope="module")
def lib():
    try:
        from paper_2605_02030_amd import uhnsw
    except ImportError as e:  # pragma: no cover - the build step makes it
        pytest.fail(f"libuhnsw.so not built: {e}")
    return uhnsw


@pytest.fixture(scope="module")
def small():
    wl = synth.make_workload(1, n=400, nq=4, d=8)
    g1, g2 = sg.build_graphs(wl, cache=False)
    assert g1.max_level >= 1 and g2.max_level >= 1
    return wl, g1, g2


def _check(lib, base, g1, g2, storage=0):
    idx, keep = lib.index_struct(base, g1, g2, storage)
    rc, msg = lib.check_index(idx)
    del keep
    return rc, msg


def test_valid_index_passes(lib, small):
    wl, g1, g2 = small
    for storage in (lib.STORE_F32, lib.STORE_BF16, lib.STORE_F16):
        assert _check(lib, wl.base, g1, g2, storage) == (lib.UHNSW_OK, "")


def _damage(g, what):
    g = copy.deepcopy(g)
    L0, L1 = g.layers[0], g.layers[1]
    if what == "M_zero":
        g.M = 0
    elif what == "M_wide":
        g.M = 33
    elif what == "edge_out_of_range":
        L0.col[3] = g.n
    elif what == "edge_negative":
        L0.col[0] = -1
    elif what == "edge_off_layer":  # layer-1 edge to a node with level 0
        L1.col[0] = int(np.flatnonzero(g.levels == 0)[0])
    elif what == "degree_above_2M":
        extra = np.arange(2 * g.M + 1, dtype=np.int32) % g.n
        L0.col = np.concatenate([extra, L0.col[L0.row_ptr[1]:]]).astype(np.int32)
        L0.row_ptr = L0.row_ptr.copy()
        L0.row_ptr[1:] += len(extra) - (L0.row_ptr[1] - L0.row_ptr[0])
    elif what == "row_ptr_not_zero":
        L0.row_ptr = L0.row_ptr + 1
    elif what == "row_ptr_decreasing":
        L0.row_ptr = L0.row_ptr.copy()
        L0.row_ptr[2] = L0.row_ptr[1] - 1
    elif what == "entry_not_on_top":
        g.entry = int(np.flatnonzero(g.levels == 0)[0])
    elif what == "entry_out_of_range":
        g.entry = g.n
    elif what == "max_level_wrong":
        g.max_level = g.max_level - 1
        g.layers = g.layers[:-1]
    elif what == "level_negative":
        g.levels = g.levels.copy()
        g.levels[5] = -1
    elif what == "nodes_unsorted":
        if len(L1.nodes) < 2:
            pytest.skip("layer 1 too small")
        L1.nodes = L1.nodes.copy()
        L1.nodes[[0, 1]] = L1.nodes[[1, 0]]
    elif what in ("dup_layer0", "dup_layer1"):  # one row lists a neighbour twice
        L = L0 if what == "dup_layer0" else L1
        r = int(np.flatnonzero(np.diff(L.row_ptr) >= 2)[0])
        L.col = L.col.copy()
        L.col[L.row_ptr[r] + 1] = L.col[L.row_ptr[r]]
    elif what in ("self_loop_layer0", "self_loop_layer1"):  # a node lists itself
        L = L0 if what == "self_loop_layer0" else L1
        r = int(np.flatnonzero(np.diff(L.row_ptr) >= 1)[0])
        L.col = L.col.copy()
        L.col[L.row_ptr[r]] = r if L.nodes is None else int(L.nodes[r])
    elif what == "nodes_count_wrong":  # drop the last node of layer 1
        L1.nodes = L1.nodes[:-1].copy()
        L1.row_ptr = L1.row_ptr[:-1].copy()
        L1.col = L1.col[:L1.row_ptr[-1]].copy()
    else:
        raise ValueError(what)
    return g


# damage -> the reason the loader must give
DAMAGES = {"M_zero": "M=0 outside", "M_wide": "M=33 outside", "edge_out_of_range": "layer 0 edge to",
           "edge_negative": "layer 0 edge to -1", "edge_off_layer": "layer 1 edge to",
           "degree_above_2M": "row 0 degree 33", "row_ptr_not_zero": "row_ptr[0] != 0",
           "row_ptr_decreasing": "row 1 degree -1", "entry_not_on_top": "not on the top layer",
           "entry_out_of_range": "entry point out of range", "max_level_wrong": "not on the top layer",
           "level_negative": "level[5] out of range", "nodes_unsorted": "not ascending",
           "nodes_count_wrong": "levels say", "dup_layer0": "twice", "dup_layer1": "twice",
           "self_loop_layer0": "lists itself", "self_loop_layer1": "lists itself"}


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("what", sorted(DAMAGES))
def test_structural_damage_refused(lib, small, what, which):
    wl, g1, g2 = small
    gs = [g1, g2]
    gs[which] = _damage(gs[which], what)
    rc, msg = _check(lib, wl.base, *gs)
    assert rc == lib.UHNSW_EINVAL, (what, msg)
    assert msg.startswith("G1" if which == 0 else "G2") and DAMAGES[what] in msg, msg


def test_base_and_sizes_refused(lib, small):
    wl, g1, g2 = small
    bad = wl.base.copy()
    bad[7, 3] = np.nan
    rc, msg = _check(lib, bad, g1, g2)
    assert rc == lib.UHNSW_EINVAL and "not finite" in msg
    bad[7, 3] = np.inf
    assert _check(lib, bad, g1, g2)[0] == lib.UHNSW_EINVAL
    rc, msg = _check(lib, wl.base, g1, g2, storage=3)
    assert rc == lib.UHNSW_EINVAL and "storage" in msg
    idx, keep = lib.index_struct(wl.base, g1, g2, variant=3)
    rc, msg = lib.check_index(idx)
    assert rc == lib.UHNSW_EINVAL and "variant" in msg
    idx.variant = lib.VARIANT_PGRAPH  # the per-p variant needs the p its graph was built for
    for gp in (0.0, 0.1, 2.5, float("nan")):
        idx.graph_p = gp
        rc, msg = lib.check_index(idx)
        assert rc == lib.UHNSW_EINVAL and "graph_p" in msg, (gp, msg)
    idx.graph_p = 0.7
    assert lib.check_index(idx) == (lib.UHNSW_OK, "")
    idx.variant = lib.VARIANT_EXT  # any structurally valid pair is accepted for either variant
    assert lib.check_index(idx) == (lib.UHNSW_OK, "")
    del keep
    wide = np.zeros((wl.n, lib.UHNSW_DMAX + 1), np.float32)
    rc, msg = _check(lib, wide, g1, g2)
    assert rc == lib.UHNSW_EINVAL and "d=" in msg
    # a graph over fewer nodes than the base: its levels say fewer rows on layer 0
    idx, keep = lib.index_struct(wl.base, g1, g2)
    idx.n = wl.n - 1
    assert lib.check_index(idx)[0] == lib.UHNSW_EINVAL
    idx.n = 0
    assert lib.check_index(idx)[0] == lib.UHNSW_EINVAL
    idx.n = wl.n
    idx.base = None
    rc, msg = lib.check_index(idx)
    assert rc == lib.UHNSW_EINVAL and "NULL" in msg
    del keep


def test_message_truncated(lib, small):
    import ctypes

    wl, g1, g2 = small
    idx, keep = lib.index_struct(wl.base, _damage(g1, "M_wide"), g2)
    buf = ctypes.create_string_buffer(b"x" * 16)
    assert lib.uhnsw_check_index(ctypes.byref(idx), buf, 8) == lib.UHNSW_EINVAL
    assert len(buf.value) == 7 and buf.raw[7:8] == b"\0" and buf.raw[8:16] == b"x" * 8
    assert lib.uhnsw_check_index(ctypes.byref(idx), None, 0) == lib.UHNSW_EINVAL
    assert lib.uhnsw_check_index(None, None, 0) == lib.UHNSW_EINVAL
    del keep


def test_files_checked_without_device(lib, small, tmp_path):
    wl, g1, g2 = small
    vp, p1, p2 = (str(tmp_path / f) for f in ("base.fbin", "g1.uhg", "g2.uhg"))
    sg.save_fbin(vp, wl.base)
    sg.save_graph_file(p1, g1)
    sg.save_graph_file(p2, g2)
    assert lib.check_index_files(vp, p1, p2) == (lib.UHNSW_OK, "")
    raw = open(p1, "rb").read()
    cases = {
        "missing": (vp, p1, str(tmp_path / "none.uhg")),
        "magic": (vp, _write(tmp_path / "magic.uhg", b"UHG2" + raw[4:]), p2),
        "truncated": (vp, _write(tmp_path / "cut.uhg", raw[:-7]), p2),
        "header": (vp, _write(tmp_path / "hdr.uhg", raw[:4] + np.int32(0).tobytes() + raw[8:]), p2),
        "short_vectors": (_write(tmp_path / "short.fbin", open(vp, "rb").read()[:-4]), p1, p2),
    }
    small_v = str(tmp_path / "small.fbin")
    sg.save_fbin(small_v, wl.base[:100])
    cases["node_count"] = (small_v, p1, p2)
    for name, args in cases.items():
        rc, msg = lib.check_index_files(*args)
        assert rc == lib.UHNSW_EIO, (name, msg)
        assert msg, name
    # a file that parses but breaks the structure is EINVAL, as from memory
    bad = _damage(g1, "edge_out_of_range")
    pb = str(tmp_path / "bad.uhg")
    sg.save_graph_file(pb, bad)
    rc, msg = lib.check_index_files(vp, pb, p2)
    assert rc == lib.UHNSW_EINVAL and msg.startswith("G1"), msg
    rc, msg = lib.check_index_files(vp, p1, p2, storage=9)
    assert rc == lib.UHNSW_EINVAL and "storage" in msg


def _write(path, data):
    with open(path, "wb") as f:
        f.write(data)
    return str(path)


def test_host_allocation_failure_is_an_error_code(small, tmp_path):
    """A host allocation that fails inside an entry point ends the call with
    UHNSW_ENOMEM and a message: no C++ exception crosses the C boundary. A
    child process caps its address space 1 GiB above what it already maps
    and asks uhnsw_check_index_files to read a 4 GiB (sparse) vector file;
    without the guard the child would end in std::terminate."""
    import os
    import subprocess
    import sys

    wl, g1, g2 = small
    vp, p1, p2 = (str(tmp_path / f) for f in ("big.fbin", "g1.uhg", "g2.uhg"))
    sg.save_graph_file(p1, g1)
    sg.save_graph_file(p2, g2)
    with open(vp, "wb") as f:
        f.truncate(4 << 30)
    child = f"""
import resource
from paper_2605_02030_amd import uhnsw
vm = next(int(l.split()[1]) * 1024 for l in open('/proc/self/status') if l.startswith('VmSize:'))
resource.setrlimit(resource.RLIMIT_AS, (vm + (1 << 30), resource.RLIM_INFINITY))
rc, msg = uhnsw.check_index_files({vp!r}, {p1!r}, {p2!r})
print(rc, msg)
"""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", child], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    rc, _, msg = r.stdout.strip().partition(" ")
    assert int(rc) == -2 and msg.startswith("uhnsw_check_index_files: host resources exhausted"), r.stdout
