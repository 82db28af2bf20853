"""CPU-side checks of the C-ABI library: it loads, it exports every entry
point include/uhnsw.h declares, and the pure host helpers behave. No HIP
device call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uhnsw.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(uhnsw_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_02030_amd import uhnsw

    return uhnsw


def test_header_declares_load_and_search_entry_points():
    names = _declared()
    for must in ("uhnsw_load_graphs", "uhnsw_search", "uhnsw_search_device", "uhnsw_create", "uhnsw_destroy",
                 "uhnsw_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in _declared():
        assert hasattr(so, name), name
    assert set(_declared()) == set(lib.EXPORTS)


def test_default_params(lib):
    p = lib.default_params()
    assert abs(p.tau - 0.92) < 1e-15 and p.cutoff == 0.0  # 0: the index's default cutoff (1.4 / 0.6)
    assert p.beam_width == 1 and p.early_abort == 1 and p.t == 0 and p.kappa == 0
    assert p.fused == 0 and p.persistent == 3 and p.graph == 0 and p.timing == 0
    q = lib.default_params(tau=0.5, beam_width=2)
    assert q.tau == 0.5 and q.beam_width == 2


def test_struct_sizes_match_header(lib):
    # uhnsw_params: double + float + 11 int32 = 56 bytes
    assert ctypes.sizeof(lib.uhnsw_params) == 56
    assert ctypes.sizeof(lib.uhnsw_graph) == 12 + 4 + 8 + 32 * 8 * 4  # M..entry, pad, level ptr, 4 arrays
    # n, d (+pad), base, storage (+pad), two graphs, variant (+pad)
    assert ctypes.sizeof(lib.uhnsw_index) == 8 + 8 + 8 + 8 + 2 * ctypes.sizeof(lib.uhnsw_graph) + 8
    assert lib.STATS_DTYPE.itemsize == 48


def test_struct_layouts_match_c(lib, tmp_path):
    """The ctypes structs against the C compiler's layout of include/uhnsw.h."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    fields = {"uhnsw_index": [f for f, _ in lib.uhnsw_index._fields_],
              "uhnsw_params": [f for f, _ in lib.uhnsw_params._fields_],
              "uhnsw_graph": ["M", "max_level", "entry_point", "level", "n_nodes", "nodes", "row_ptr", "col"],
              "uhnsw_serve_config": [f for f, _ in lib.uhnsw_serve_config._fields_],
              "uhnsw_stats": [f for f, _ in lib.uhnsw_stats._fields_],
              "uhnsw_serve_result": [f for f, _ in lib.uhnsw_serve_result._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "uhnsw.h"', "int main(void) {"]
    for st, fl in fields.items():
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        st, f, v = line.split()
        cls = getattr(lib, st)
        got = ctypes.sizeof(cls) if f == "size" else getattr(cls, f).offset
        assert got == int(v), line


def test_null_arguments_rejected_without_device(lib):
    # these return before touching the HIP runtime
    assert lib.uhnsw_create(0, None) == lib.UHNSW_EINVAL
    assert lib.uhnsw_load_graphs(None, None) == lib.UHNSW_EINVAL
    assert lib.uhnsw_reset(None) == lib.UHNSW_EINVAL
    assert lib.uhnsw_search(None, None, 0, None, None, None, None, 0, None, None, None) == lib.UHNSW_EINVAL
    lib.uhnsw_destroy(None)


def test_device_arguments_checked_before_the_call(lib):
    """The device entry points take raw pointers, so the binding refuses what
    the kernels would misread -- host tensors, wrong dtypes, non-contiguous
    views, short outputs, half of the candidate pair -- with TypeError /
    ValueError, before any HIP call."""
    import torch

    nq, d = 4, 8
    q, p = torch.zeros((nq, d)), torch.ones(nq)
    k, ef = torch.full((nq,), 10, dtype=torch.int32), torch.full((nq,), 64, dtype=torch.int32)
    with pytest.raises(ValueError, match="device tensor"):
        lib._check_device_args(q, p, k, ef)
    with pytest.raises(TypeError, match="torch tensor"):
        lib._check_device_args(q.numpy(), p, k, ef)

    # the checks after the device test, on host tensors made to report
    # is_cuda (the checks read attributes only; nothing is launched)
    had = "is_cuda" in torch.Tensor.__dict__
    orig = torch.Tensor.__dict__.get("is_cuda")
    try:
        torch.Tensor.is_cuda = property(lambda self: True)
        ok = dict(ids=torch.zeros((nq, 10), dtype=torch.int64), dists=torch.zeros((nq, 10)),
                  stats=torch.zeros((nq, lib.STATS_WORDS), dtype=torch.int32))
        lib._check_device_args(q, p, k, ef, **ok)
        bad = [
            (dict(k=k.long()), TypeError, "k: dtype"),
            (dict(p=p.double()), TypeError, "p: dtype"),
            (dict(q=q.t()), ValueError, "queries: must be contiguous"),
            (dict(ef=ef[:2]), ValueError, "ef: 2 elements"),
            (dict(ids=ok["ids"][:2]), ValueError, "ids: .* fewer than 4 rows"),
            (dict(dists=torch.zeros((nq, 5))), ValueError, "different k_stride"),
            (dict(stats=torch.zeros((nq, 2), dtype=torch.int32)), ValueError, "stats"),
            (dict(cand_ids=torch.zeros((nq, 60), dtype=torch.int32)), ValueError, "both or neither"),
        ]
        for change, exc, msg in bad:
            args = dict(q=q, p=p, k=k, ef=ef, **ok)
            args.update(change)
            with pytest.raises(exc, match=msg):
                lib._check_device_args(args.pop("q"), args.pop("p"), args.pop("k"), args.pop("ef"), **args)
    finally:
        if had:
            torch.Tensor.is_cuda = orig
        else:
            del torch.Tensor.is_cuda
    assert not torch.zeros(1).is_cuda
