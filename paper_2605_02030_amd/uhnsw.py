"""ctypes binding of libuhnsw (include/uhnsw.h): the same entry points, with
argument marshalling only. Every step of the query path runs in the HIP
kernels of libuhnsw.so; there is no CPU fallback. Importing this module on a
tree without the built library raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuhnsw.so")

UHNSW_OK, UHNSW_EINVAL, UHNSW_ENOMEM, UHNSW_EDEVICE = 0, -1, -2, -3
UHNSW_ESTATE, UHNSW_EIO, UHNSW_EBUSY, UHNSW_EUNSUPPORTED = -4, -5, -6, -7
UHNSW_MAX_LAYERS, UHNSW_KMAX, UHNSW_EFMAX, UHNSW_DMAX = 32, 256, 2048, 1024
UHNSW_NOALLOC_SCRATCH_BYTES = 64 << 20
STORE_F32, STORE_BF16, STORE_F16 = 0, 1, 2
UHNSW_QBAD, UHNSW_QCAP = 1, 2
UHNSW_TUNE_BEAM, UHNSW_TUNE_PIPELINED = 1, 2
VARIANT_STD, VARIANT_EXT, VARIANT_PGRAPH = 0, 1, 2
METRIC_L1, METRIC_L2, METRIC_L05, METRIC_LP = 1, 2, 3, 4

EXPORTS = ("uhnsw_default_params", "uhnsw_create", "uhnsw_destroy", "uhnsw_last_error", "uhnsw_load_graphs",
           "uhnsw_search", "uhnsw_search_device", "uhnsw_get_layout", "uhnsw_last_timing", "uhnsw_device_info",
           "uhnsw_autotune", "uhnsw_graph_captures", "uhnsw_serve_default_config", "uhnsw_serve_start",
           "uhnsw_serve_submit", "uhnsw_serve_poll", "uhnsw_serve_info", "uhnsw_serve_drive", "uhnsw_serve_stop",
           "uhnsw_probe_gather", "uhnsw_probe_transcendental", "uhnsw_load_graph_files", "uhnsw_check_index",
           "uhnsw_check_index_files", "uhnsw_reset", "uhnsw_last_timing_split", "uhnsw_search_device_noalloc",
           "uhnsw_build_graph", "uhnsw_built_graph_view", "uhnsw_built_graph_free")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2605_02030_amd.build` "
                      "(or __graft_entry__.build()) first")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I32, _I64 = ctypes.c_int32, ctypes.c_int64


class uhnsw_graph(ctypes.Structure):
    _fields_ = [("M", _I32), ("max_level", _I32), ("entry_point", _I32), ("level", _P),
                ("n_nodes", _I64 * UHNSW_MAX_LAYERS), ("nodes", _P * UHNSW_MAX_LAYERS),
                ("row_ptr", _P * UHNSW_MAX_LAYERS), ("col", _P * UHNSW_MAX_LAYERS)]


class uhnsw_index(ctypes.Structure):
    _fields_ = [("n", _I64), ("d", _I32), ("base", _P), ("storage", _I32), ("graphs", uhnsw_graph * 2),
                ("variant", _I32), ("graph_p", ctypes.c_float)]


class uhnsw_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("cutoff", ctypes.c_float), ("t", _I32), ("kappa", _I32),
                ("beam_width", _I32), ("early_abort", _I32), ("visited_slots", _I32),
                ("waves_per_block", _I32), ("persistent", _I32), ("timing", _I32), ("fused", _I32),
                ("graph", _I32), ("waves_per_cu", _I32)]


class uhnsw_stats(ctypes.Structure):
    _fields_ = [(f, _I32) for f in ("graph", "n_b", "n_exp", "n_p", "batches", "nc", "flags", "entry0")] + \
               [("t_begin", ctypes.c_uint32), ("t_end", ctypes.c_uint32), ("n_up", _I32), ("n_cut", _I32)]


class uhnsw_serve_config(ctypes.Structure):
    _fields_ = [("k_max", _I32), ("ef_max", _I32), ("max_inflight", _I32), ("max_batch", _I32),
                ("streams", _I32), ("reserved", _I32), ("hbm_budget", _I64), ("params", uhnsw_params)]


class uhnsw_serve_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", _I32), ("nres", _I32), ("submit_us", ctypes.c_double),
                ("launch_us", ctypes.c_double), ("done_us", ctypes.c_double), ("stats", uhnsw_stats),
                ("ids", _I64 * UHNSW_KMAX), ("dists", ctypes.c_float * UHNSW_KMAX)]


STATS_FIELDS = ("graph", "n_b", "n_exp", "n_p", "batches", "nc", "flags", "entry0", "t_begin", "t_end", "n_up",
                "n_cut")
STATS_DTYPE = np.dtype([(f, np.int32) for f in STATS_FIELDS[:8]] + [(f, np.uint32) for f in STATS_FIELDS[8:10]]
                       + [("n_up", np.int32), ("n_cut", np.int32)])
STATS_WORDS = len(STATS_FIELDS)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


uhnsw_default_params = _sig("uhnsw_default_params", None, [_P])
uhnsw_create = _sig("uhnsw_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)])
uhnsw_destroy = _sig("uhnsw_destroy", None, [_P])
uhnsw_last_error = _sig("uhnsw_last_error", ctypes.c_char_p, [_P])
uhnsw_load_graphs = _sig("uhnsw_load_graphs", ctypes.c_int, [_P, _P])
uhnsw_reset = _sig("uhnsw_reset", ctypes.c_int, [_P])
uhnsw_search = _sig("uhnsw_search", ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _P, _I32, _P, _P, _P])
uhnsw_search_device = _sig("uhnsw_search_device", ctypes.c_int,
                           [_P, _P, _I64, _P, _P, _P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _I32, _P])
uhnsw_search_device_noalloc = _sig("uhnsw_search_device_noalloc", ctypes.c_int,
                                   [_P, _P, _I64, _P, _P, _P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _I32, _P])
uhnsw_get_layout = _sig("uhnsw_get_layout", ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)])
uhnsw_autotune = _sig("uhnsw_autotune", ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _I32, _I32, _P, _P])
uhnsw_graph_captures = _sig("uhnsw_graph_captures", ctypes.c_int, [_P, ctypes.POINTER(_I64)])
uhnsw_serve_default_config = _sig("uhnsw_serve_default_config", None, [_P])
uhnsw_serve_start = _sig("uhnsw_serve_start", ctypes.c_int, [_P, _P, ctypes.POINTER(_P)])
uhnsw_serve_submit = _sig("uhnsw_serve_submit", ctypes.c_int, [_P, _P, ctypes.c_float, _I32, _I32, ctypes.c_uint64])
uhnsw_serve_poll = _sig("uhnsw_serve_poll", ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(_I32)])
uhnsw_serve_info = _sig("uhnsw_serve_info", ctypes.c_int, [_P, _P])
uhnsw_serve_drive = _sig("uhnsw_serve_drive", ctypes.c_int,
                         [_P, _I64, _P, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P])
uhnsw_serve_stop = _sig("uhnsw_serve_stop", ctypes.c_int, [_P])
uhnsw_device_info = _sig("uhnsw_device_info", ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)])
uhnsw_last_timing = _sig("uhnsw_last_timing", ctypes.c_int,
                         [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)])
uhnsw_last_timing_split = _sig("uhnsw_last_timing_split", ctypes.c_int,
                               [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float)])
uhnsw_probe_gather = _sig("uhnsw_probe_gather", ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_double)])
uhnsw_load_graph_files = _sig("uhnsw_load_graph_files", ctypes.c_int,
                              [_P, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, _I32, _I32])
uhnsw_probe_transcendental = _sig("uhnsw_probe_transcendental", ctypes.c_int,
                                  [_P, ctypes.POINTER(ctypes.c_double)])
uhnsw_check_index = _sig("uhnsw_check_index", ctypes.c_int, [_P, ctypes.c_char_p, _I32])
uhnsw_check_index_files = _sig("uhnsw_check_index_files", ctypes.c_int,
                               [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, _I32, _I32, ctypes.c_char_p,
                                _I32])


uhnsw_build_graph = _sig("uhnsw_build_graph", ctypes.c_int,
                         [_P, _P, _I64, _I32, _I32, ctypes.c_float, _I32, _I32, ctypes.c_uint64, _I32,
                          ctypes.POINTER(_P)])
uhnsw_built_graph_view = _sig("uhnsw_built_graph_view", ctypes.c_int,
                              [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)])
uhnsw_built_graph_free = _sig("uhnsw_built_graph_free", None, [_P])


class UhnswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"uhnsw error {code}: {msg}")
        self.code = code


def default_params(**kw) -> uhnsw_params:
    p = uhnsw_params()
    uhnsw_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _graph_struct(g, keep):
    s = uhnsw_graph()
    s.M = int(g.M)
    s.max_level = int(g.max_level)
    s.entry_point = int(g.entry)
    lv = np.ascontiguousarray(g.levels, np.int8)
    keep.append(lv)
    s.level = lv.ctypes.data
    for l, L in enumerate(g.layers):
        rp = np.ascontiguousarray(L.row_ptr, np.int64)
        col = np.ascontiguousarray(L.col, np.int32)
        if col.size == 0:
            col = np.zeros(1, np.int32)
        keep += [rp, col]
        s.row_ptr[l] = rp.ctypes.data
        s.col[l] = col.ctypes.data
        if l == 0:
            s.n_nodes[l] = len(rp) - 1
        else:
            nodes = np.ascontiguousarray(L.nodes, np.int32)
            keep.append(nodes)
            s.nodes[l] = nodes.ctypes.data
            s.n_nodes[l] = nodes.shape[0]
    return s


def index_struct(base, g1, g2, storage: int = STORE_F32, variant: int = VARIANT_STD, graph_p: float = 0.0):
    """The uhnsw_index for (base, g1, g2) and the arrays it points into (keep
    them alive while the struct is used). With VARIANT_EXT, g1 / g2 are
    G_0.5 / G_1; with VARIANT_PGRAPH g1 is G_p built for graph_p."""
    base = np.ascontiguousarray(base, np.float32)
    keep = [base]
    idx = uhnsw_index()
    idx.n, idx.d = base.shape
    idx.base = base.ctypes.data
    idx.storage = storage
    idx.variant = variant
    idx.graph_p = float(graph_p)
    idx.graphs[0] = _graph_struct(g1, keep)
    idx.graphs[1] = _graph_struct(g2, keep)
    return idx, keep


def check_index(idx) -> tuple[int, str]:
    """uhnsw_check_index: (return code, reason) with no context or device."""
    msg = ctypes.create_string_buffer(512)
    rc = uhnsw_check_index(ctypes.byref(idx), msg, len(msg))
    return rc, msg.value.decode()


def check_index_files(vec_path: str, g1_path: str, g2_path: str, storage: int = STORE_F32,
                      variant: int = VARIANT_STD) -> tuple[int, str]:
    """uhnsw_check_index_files: (return code, reason) with no context or device."""
    msg = ctypes.create_string_buffer(512)
    rc = uhnsw_check_index_files(vec_path.encode(), g1_path.encode(), g2_path.encode(), storage, variant, msg,
                                 len(msg))
    return rc, msg.value.decode()


def _stream_handle(stream):
    """A raw hipStream_t from a torch stream, an int, or None (torch's
    current stream)."""
    import torch

    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _check_device_args(queries, p, k, ef, ids=None, dists=None, stats=None, cand_ids=None, cand_keys=None):
    """The device entry points take raw pointers: refuse host tensors, wrong
    dtypes, non-contiguous views and short outputs here (TypeError /
    ValueError) rather than hand the kernels a pointer they would misread."""
    import torch

    def need(t, name, dtype, rows=None, words=None):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: a torch tensor is required")
        if not t.is_cuda:
            raise ValueError(f"{name}: must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if t.dtype != dtype:
            raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
        if rows is not None and (t.dim() < 1 or t.shape[0] < rows):
            raise ValueError(f"{name}: {tuple(t.shape)} has fewer than {rows} rows")
        if words is not None and t.numel() < words:
            raise ValueError(f"{name}: {t.numel()} elements, at least {words} needed")

    need(queries, "queries", torch.float32)
    if queries.dim() != 2:
        raise ValueError("queries: (nq, d) expected")
    nq = queries.shape[0]
    for t, name, dt in ((p, "p", torch.float32), (k, "k", torch.int32), (ef, "ef", torch.int32)):
        need(t, name, dt, words=nq)
    for t, name, dt in ((ids, "ids", torch.int64), (dists, "dists", torch.float32)):
        if t is not None:
            need(t, name, dt, rows=nq)
            if t.dim() != 2:
                raise ValueError(f"{name}: (nq, k_stride) expected")
    if ids is not None and dists is not None and ids.shape[1] != dists.shape[1]:
        raise ValueError("ids and dists: different k_stride")
    if stats is not None:
        need(stats, "stats", torch.int32, words=nq * STATS_WORDS)
    if (cand_ids is None) != (cand_keys is None):
        raise ValueError("cand_ids and cand_keys: give both or neither")
    if cand_ids is not None:
        need(cand_ids, "cand_ids", torch.int32, rows=nq)
        need(cand_keys, "cand_keys", torch.float32, rows=nq)
        if cand_ids.dim() != 2 or cand_ids.shape != cand_keys.shape:
            raise ValueError("cand_ids / cand_keys: (nq, c_stride) each expected")


class Context:
    """One libuhnsw context on one HIP device (owns the resident index)."""

    def __init__(self, device: int = 0):
        h = _P()
        rc = uhnsw_create(device, ctypes.byref(h))
        if rc != UHNSW_OK:
            raise UhnswError(rc, uhnsw_last_error(None).decode())
        self.h = h
        self.n = self.d = 0

    def close(self, _destroy=uhnsw_destroy):  # bound early: usable during interpreter shutdown
        """Stop the servers still running on this context, then free it."""
        for srv in list(getattr(self, "_servers", ())):
            srv.stop()
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != UHNSW_OK:
            raise UhnswError(rc, uhnsw_last_error(self.h).decode())

    def load_graphs(self, base, g1, g2, storage: int = STORE_F32, variant: int = VARIANT_STD,
                    graph_p: float = 0.0) -> None:
        """base: (n, d) FP32; g1 / g2: graphs with M, max_level, entry, levels,
        layers[l].nodes / row_ptr / col (G1 under L1, G2 under L2; with
        VARIANT_EXT, G_0.5 under L0.5 and G_1 under L1; with VARIANT_PGRAPH,
        G_p built for graph_p and a graph walked under L2)."""
        idx, keep = index_struct(base, g1, g2, storage, variant, graph_p)
        self._check(uhnsw_load_graphs(self.h, ctypes.byref(idx)))
        self.n, self.d = int(idx.n), int(idx.d)
        del keep

    def reset(self) -> None:
        """uhnsw_reset: clear a failed state (the loaded index stays)."""
        self._check(uhnsw_reset(self.h))

    def layout(self):
        g, v = _I32(), _I32()
        self._check(uhnsw_get_layout(self.h, ctypes.byref(g), ctypes.byref(v)))
        return g.value, v.value

    def search(self, queries, p, k, ef, params: uhnsw_params | None = None, k_stride: int | None = None):
        """Host arrays in, host arrays out (synchronous)."""
        queries = np.ascontiguousarray(queries, np.float32)
        if queries.ndim != 2 or (self.d and queries.shape[1] != self.d):
            raise ValueError(f"queries: (nq, {self.d}) expected, got {queries.shape}")
        nq = queries.shape[0]
        p = np.ascontiguousarray(p, np.float32)
        k = np.ascontiguousarray(k, np.int32)
        ef = np.ascontiguousarray(ef, np.int32)
        for name, a in (("p", p), ("k", k), ("ef", ef)):
            if a.ndim != 1 or a.shape[0] != nq:  # the library reads one value per query
                raise ValueError(f"{name}: {a.shape}, expected ({nq},)")
        ks = int(k_stride if k_stride is not None else (k.max() if nq else 1))
        ids = np.empty((nq, ks), np.int64)
        dists = np.empty((nq, ks), np.float32)
        stats = np.zeros(nq, STATS_DTYPE)
        prm = ctypes.byref(params) if params is not None else None
        self._check(uhnsw_search(self.h, queries.ctypes.data, nq, p.ctypes.data, k.ctypes.data, ef.ctypes.data,
                                 prm, ks, ids.ctypes.data, dists.ctypes.data, stats.ctypes.data))
        return ids, dists, stats

    def search_device(self, queries, p, k, ef, k_max: int, ef_max: int, ids, dists, stats=None,
                      cand_ids=None, cand_keys=None, params: uhnsw_params | None = None, stream=None):
        """torch device tensors in and out; asynchronous on ``stream`` (torch
        stream or raw hipStream_t int; default: torch's current stream)."""
        _check_device_args(queries, p, k, ef, ids, dists, stats, cand_ids, cand_keys)
        stream = _stream_handle(stream)
        nq = queries.shape[0]
        ks = ids.shape[1]
        cs = cand_ids.shape[1] if cand_ids is not None else 0
        prm = ctypes.byref(params) if params is not None else None
        self._check(uhnsw_search_device(
            self.h, queries.data_ptr(), nq, p.data_ptr(), k.data_ptr(), ef.data_ptr(), int(k_max), int(ef_max),
            prm, ks, ids.data_ptr(), dists.data_ptr(), stats.data_ptr() if stats is not None else None,
            cand_ids.data_ptr() if cand_ids is not None else None,
            cand_keys.data_ptr() if cand_keys is not None else None, cs, stream))

    def search_device_noalloc(self, queries, p, k, ef, k_max: int, ef_max: int, ids, dists, stats=None,
                              cand_ids=None, cand_keys=None, params: uhnsw_params | None = None, stream=None):
        """search_device without any allocation (scratch from the device's
        fixed region; see include/uhnsw.h)."""
        _check_device_args(queries, p, k, ef, ids, dists, stats, cand_ids, cand_keys)
        stream = _stream_handle(stream)
        cs = cand_ids.shape[1] if cand_ids is not None else 0
        prm = ctypes.byref(params) if params is not None else None
        self._check(uhnsw_search_device_noalloc(
            self.h, queries.data_ptr(), queries.shape[0], p.data_ptr(), k.data_ptr(), ef.data_ptr(), int(k_max),
            int(ef_max), prm, ids.shape[1], ids.data_ptr(), dists.data_ptr(),
            stats.data_ptr() if stats is not None else None, cand_ids.data_ptr() if cand_ids is not None else None,
            cand_keys.data_ptr() if cand_keys is not None else None, cs, stream))

    def autotune(self, queries, p, k, ef, k_max: int, ef_max: int, params: uhnsw_params | None = None,
                 allow_beam: bool = False, pipelined: bool = False, stream=None) -> uhnsw_params:
        """Time the execution knobs on these device tensors; returns tuned params.
        allow_beam: also choose the beam width (changes the walk); pipelined:
        time back-to-back launches with two in flight."""
        _check_device_args(queries, p, k, ef)
        stream = _stream_handle(stream)
        flags = (UHNSW_TUNE_BEAM if allow_beam else 0) | (UHNSW_TUNE_PIPELINED if pipelined else 0)
        prm = params if params is not None else default_params()
        prm = uhnsw_params.from_buffer_copy(prm)
        self._check(uhnsw_autotune(self.h, queries.data_ptr(), queries.shape[0], p.data_ptr(), k.data_ptr(),
                                   ef.data_ptr(), int(k_max), int(ef_max), flags, ctypes.byref(prm),
                                   stream))
        return prm

    def graph_captures(self) -> int:
        n = _I64()
        self._check(uhnsw_graph_captures(self.h, ctypes.byref(n)))
        return n.value

    def device_info(self):
        cus, khz = _I32(), _I32()
        self._check(uhnsw_device_info(self.h, ctypes.byref(cus), ctypes.byref(khz)))
        return cus.value, khz.value

    def load_graph_files(self, vec_path: str, g1_path: str, g2_path: str, storage: int = STORE_F32,
                         variant: int = VARIANT_STD):
        """Load an index from a .fbin vector file and two UHG1 graph files."""
        self._check(uhnsw_load_graph_files(self.h, os.fsencode(vec_path), os.fsencode(g1_path),
                                           os.fsencode(g2_path), int(storage), int(variant)))
        self.n, self.d = (int(x) for x in np.fromfile(vec_path, np.int32, 2))

    def probe_gather(self, row_bytes: int) -> float:
        """GB/s of random row gathers with the walk's access pattern (ceiling probe)."""
        v = ctypes.c_double()
        self._check(uhnsw_probe_gather(self.h, int(row_bytes), ctypes.byref(v)))
        return v.value

    def probe_transcendental(self) -> float:
        """v_exp + v_log lane operations per second (ceiling probe)."""
        v = ctypes.c_double()
        self._check(uhnsw_probe_transcendental(self.h, ctypes.byref(v)))
        return v.value

    def last_timing(self):
        w, v = ctypes.c_float(), ctypes.c_float()
        self._check(uhnsw_last_timing(self.h, ctypes.byref(w), ctypes.byref(v)))
        return w.value, v.value

    def last_timing_split(self):
        """(pre-pass ms, walk kernel ms, verification ms) of the last timed search."""
        a, w, v = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        self._check(uhnsw_last_timing_split(self.h, ctypes.byref(a), ctypes.byref(w), ctypes.byref(v)))
        return a.value, w.value, v.value


class BuiltLayer:
    def __init__(self, nodes, row_ptr, col):
        self.nodes, self.row_ptr, self.col = nodes, row_ptr, col


class BuiltGraph:
    """A graph made by uhnsw_build_graph, copied into numpy arrays (the
    fields load_graphs reads: M, max_level, entry, levels, layers)."""

    def __init__(self, view: uhnsw_graph, n: int, metric: int, seconds: float, batches: int):
        self.metric, self.n, self.M = metric, n, int(view.M)
        self.max_level, self.entry = int(view.max_level), int(view.entry_point)
        self.seconds, self.batches = seconds, batches
        self.levels = np.ctypeslib.as_array(ctypes.cast(view.level, ctypes.POINTER(ctypes.c_int8)), (n,)).copy()
        self.layers = []
        for l in range(self.max_level + 1):
            nl = int(view.n_nodes[l])
            rp = np.ctypeslib.as_array(ctypes.cast(view.row_ptr[l], ctypes.POINTER(_I64)), (nl + 1,)).copy()
            ne = int(rp[-1])
            col = np.ctypeslib.as_array(ctypes.cast(view.col[l], ctypes.POINTER(_I32)), (max(ne, 1),))[:ne].copy()
            nodes = None
            if l:
                nodes = np.ctypeslib.as_array(ctypes.cast(view.nodes[l], ctypes.POINTER(_I32)), (nl,)).copy()
            self.layers.append(BuiltLayer(nodes, rp, col))

    @property
    def M0(self) -> int:
        return 2 * self.M


def build_graph(ctx: "Context", base, metric: int, M: int = 16, ef_construction: int = 200, seed: int = 0,
                batch_max: int = 1024, metric_p: float = 0.0) -> BuiltGraph:
    """uhnsw_build_graph on ctx's device: one HNSW graph of `base` under
    `metric` (METRIC_L1, METRIC_L2, METRIC_L05, or METRIC_LP with metric_p)."""
    base = np.ascontiguousarray(base, np.float32)
    n, d = base.shape
    h = _P()
    ctx._check(uhnsw_build_graph(ctx.h, base.ctypes.data, n, d, int(metric), float(metric_p), int(M),
                                 int(ef_construction), int(seed), int(batch_max), ctypes.byref(h)))
    try:
        view = uhnsw_graph()
        sec, nb = ctypes.c_double(), _I64()
        ctx._check(uhnsw_built_graph_view(h, ctypes.byref(view), ctypes.byref(sec), ctypes.byref(nb)))
        return BuiltGraph(view, n, metric, sec.value, nb.value)
    finally:
        uhnsw_built_graph_free(h)


class Server:
    """Continuous-batching server on a Context (include/uhnsw.h, serving form)."""

    def __init__(self, ctx: Context, **cfg):
        c = uhnsw_serve_config()
        uhnsw_serve_default_config(ctypes.byref(c))
        for key, val in cfg.items():
            if key == "params":
                c.params = val
            else:
                setattr(c, key, val)
        h = _P()
        rc = uhnsw_serve_start(ctx.h, ctypes.byref(c), ctypes.byref(h))
        if rc != UHNSW_OK:
            raise UhnswError(rc, "uhnsw_serve_start: " + uhnsw_last_error(ctx.h).decode())
        self.h, self.ctx, self.d, self.cfg = h, ctx, ctx.d, c
        if not hasattr(ctx, "_servers"):
            ctx._servers = weakref.WeakSet()
        ctx._servers.add(self)

    def submit(self, q, p, k, ef, tag) -> int:
        q = np.ascontiguousarray(q, np.float32).ravel()
        if q.size != self.d:  # the library copies d floats
            raise ValueError(f"query of {q.size} values, the index has d = {self.d}")
        return uhnsw_serve_submit(self.h, q.ctypes.data, float(p), int(k), int(ef), int(tag))

    def poll(self, max_n=256):
        buf = (uhnsw_serve_result * max_n)()
        n = _I32()
        rc = uhnsw_serve_poll(self.h, buf, max_n, ctypes.byref(n))
        if rc != UHNSW_OK:
            raise UhnswError(rc, "uhnsw_serve_poll failed")
        return [buf[i] for i in range(n.value)]

    def info(self):
        a = np.zeros(10, np.int64)
        uhnsw_serve_info(self.h, a.ctypes.data)
        return dict(zip(("slots", "free", "pending", "batches", "completed", "max_overlap", "max_batch",
                         "streams", "waves_per_cu", "cus"), a.tolist()))

    def drive(self, queries, p, k, ef, arrival_us, with_stats=False, out_k=None, qidx=None):
        """Submit on the given schedule, return (ids, dists, status, submit_us, launch_us, done_us)
        (and the per-query stats as a STATS_DTYPE array when with_stats); ids /
        dists hold the first out_k (default: the server's k_max) entries of each
        row. With qidx, arrival i carries queries[qidx[i]] (p, k, ef, arrival_us
        are per arrival)."""
        queries = np.ascontiguousarray(queries, np.float32)
        if queries.ndim != 2 or queries.shape[1] != self.d:
            raise ValueError(f"queries: (m, {self.d}) expected, got {queries.shape}")
        n = queries.shape[0] if qidx is None else len(qidx)
        if qidx is not None:
            qidx = np.ascontiguousarray(qidx, np.int32)
            if n and (qidx.min() < 0 or qidx.max() >= queries.shape[0]):
                raise ValueError("qidx: a row index outside queries")
        p = np.ascontiguousarray(p, np.float32)
        k = np.ascontiguousarray(k, np.int32)
        ef = np.ascontiguousarray(ef, np.int32)
        arr = np.ascontiguousarray(arrival_us, np.float64)
        for name, a in (("p", p), ("k", k), ("ef", ef), ("arrival_us", arr)):
            if a.ndim != 1 or a.shape[0] != n:  # the library reads one value per arrival
                raise ValueError(f"{name}: {a.shape}, expected ({n},)")
        ok = int(out_k or self.cfg.k_max)
        ids = np.empty((n, ok), np.int64)
        dists = np.empty((n, ok), np.float32)
        st = np.zeros(n, STATS_DTYPE) if with_stats else None
        times = np.empty((n, 3), np.float64)
        status = np.empty(n, np.int32)
        rc = uhnsw_serve_drive(self.h, n, queries.ctypes.data, qidx.ctypes.data if qidx is not None else None,
                               p.ctypes.data, k.ctypes.data, ef.ctypes.data, arr.ctypes.data, ok, ids.ctypes.data, dists.ctypes.data,
                               st.ctypes.data if with_stats else None, times.ctypes.data, status.ctypes.data)
        if rc != UHNSW_OK:
            raise UhnswError(rc, "uhnsw_serve_drive failed")
        out = (ids, dists, status, times[:, 0], times[:, 1], times[:, 2])
        return out + (st,) if with_stats else out

    def stop(self):
        if getattr(self, "h", None):
            rc = uhnsw_serve_stop(self.h)
            self.h = None
            if rc != UHNSW_OK:
                raise UhnswError(rc, "server ended with an error: " + uhnsw_last_error(self.ctx.h).decode())

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
