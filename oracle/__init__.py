"""CPU oracle for the U-HNSW query path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``oracle.c`` (plain C,
FP64 for L_p, the paper's Algorithm 1 step by step) through ctypes and shares
no code with the GPU library ``paper_2605_02030_amd``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")

F32, BF16, F16 = 0, 1, 2
L1, L2, L05, LP = 1, 2, 3, 4  # base metrics of the walk (L05: sum sqrt|x - q|; LP: sum |x - q|^mp)
VARIANT_STD, VARIANT_EXT, VARIANT_PGRAPH = 0, 1, 2
MAXL = 32
_lib = None


def build_lib(force: bool = True) -> str:
    """Compile ``oracle/_oracle.so`` (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                        "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OrcGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("max_level", ctypes.c_int), ("entry", ctypes.c_int32),
                ("max_deg0", ctypes.c_int),
                ("nnodes", ctypes.c_int64 * MAXL), ("nodes", ctypes.c_void_p * MAXL),
                ("row_ptr", ctypes.c_void_p * MAXL), ("col", ctypes.c_void_p * MAXL)]


class OrcData(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int), ("base", ctypes.c_void_p),
                ("walk_storage", ctypes.c_int), ("walk_base", ctypes.c_void_p)]


class OrcParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("cutoff", ctypes.c_float), ("t_param", ctypes.c_int),
                ("kappa", ctypes.c_int), ("w", ctypes.c_int), ("early_abort", ctypes.c_int),
                ("g", ctypes.c_int), ("v", ctypes.c_int), ("cache_slots", ctypes.c_int), ("variant", ctypes.c_int),
                ("walk_p", ctypes.c_double)]


class OrcStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("graph", "n_b", "n_exp", "n_p", "batches", "nc", "nres", "m",
                                                         "entry0")]


STATS_DTYPE = np.dtype([(f, np.int32) for f in ("graph", "n_b", "n_exp", "n_p", "batches", "nc", "nres", "m",
                                                 "entry0")])

_P = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        L = ctypes.CDLL(_LIB)
        L.orc_lp_sum.restype = ctypes.c_double
        L.orc_lp_sum.argtypes = [_P, _P, ctypes.c_int, ctypes.c_double]
        L.orc_lp_dist.restype = ctypes.c_double
        L.orc_lp_dist.argtypes = [_P, _P, ctypes.c_int, ctypes.c_double]
        L.orc_bruteforce.argtypes = [_P, ctypes.c_int64, ctypes.c_int, _P, ctypes.c_int64, _P, ctypes.c_int,
                                     _P, _P, ctypes.c_int]
        L.orc_convert.argtypes = [_P, ctypes.c_int64, ctypes.c_int, _P]
        L.orc_bf16_to_f32.restype = ctypes.c_float
        L.orc_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.orc_f16_to_f32.restype = ctypes.c_float
        L.orc_f16_to_f32.argtypes = [ctypes.c_uint16]
        L.orc_base_dist.restype = ctypes.c_float
        L.orc_base_dist.argtypes = [_P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int]
        L.orc_m_of.restype = ctypes.c_int
        L.orc_m_of.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_knn_search.restype = ctypes.c_int
        L.orc_knn_search.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P]
        L.orc_verify.restype = ctypes.c_int
        L.orc_verify.argtypes = [_P, _P, ctypes.c_float, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]
        L.orc_query_batch.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int,
                                      _P, _P, _P, ctypes.c_int, _P, _P, _P, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ------------------------------------------------------------------ L_p
def lp_sum(x, q, p) -> float:
    x, q = _f32(x), _f32(q)
    return _load().orc_lp_sum(_ptr(x), _ptr(q), x.shape[-1], float(p))


def lp_dist(x, q, p) -> float:
    x, q = _f32(x), _f32(q)
    return _load().orc_lp_dist(_ptr(x), _ptr(q), x.shape[-1], float(p))


def bruteforce(base, queries, p, K, threads=0):
    """Exact top-K by (S_p, id) under L_p for each query; returns (ids int32, S float64)."""
    base, queries = _f32(base), _f32(queries)
    p = _f32(np.broadcast_to(np.asarray(p, np.float32), (queries.shape[0],)))
    nq = queries.shape[0]
    ids = np.empty((nq, K), np.int32)
    S = np.empty((nq, K), np.float64)
    _load().orc_bruteforce(_ptr(base), base.shape[0], base.shape[1], _ptr(queries), nq, _ptr(p), K,
                           _ptr(ids), _ptr(S), threads)
    return ids, S


# ------------------------------------------------------------- storage
def convert(x, storage):
    """FP32 -> bfloat16 / binary16 bit patterns (uint16), round to nearest even."""
    x = _f32(x)
    out = np.empty(x.shape, np.uint16)
    _load().orc_convert(_ptr(x), x.size, storage, _ptr(out))
    return out


def widen(h, storage):
    L = _load()
    f = L.orc_bf16_to_f32 if storage == BF16 else L.orc_f16_to_f32
    flat = np.ascontiguousarray(h, np.uint16).ravel()
    return np.array([f(int(v)) for v in flat], np.float32).reshape(np.shape(h))


def base_dist(x, q, metric, g, v, storage=F32, mp=0.0) -> float:
    """The walk's FP32 key of row x for query q (mp: the p of metric LP)."""
    x = np.ascontiguousarray(x) if storage != F32 else _f32(x)
    q = _f32(q)
    return _load().orc_base_dist(_ptr(x), storage, _ptr(q), q.shape[0], metric, float(mp), g, v)


def m_of(tau, K) -> int:
    return _load().orc_m_of(float(tau), int(K))


# -------------------------------------------------------------- graphs
class Graph:
    """ctypes view of a :class:`synth.graphs.Graph` (keeps the arrays alive)."""

    def __init__(self, g):
        self.src = g
        s = OrcGraph()
        s.n = g.n
        s.max_level = g.max_level
        s.entry = g.entry
        rp0 = g.layers[0].row_ptr
        s.max_deg0 = int(np.diff(rp0).max()) if g.n else 0
        self._keep = []
        for l, L in enumerate(g.layers):
            rp = np.ascontiguousarray(L.row_ptr, np.int64)
            col = np.ascontiguousarray(L.col, np.int32)
            if col.size == 0:
                col = np.zeros(1, np.int32)
            self._keep += [rp, col]
            s.row_ptr[l] = rp.ctypes.data
            s.col[l] = col.ctypes.data
            if l == 0:
                s.nnodes[l] = g.n
            else:
                nodes = np.ascontiguousarray(L.nodes, np.int32)
                self._keep.append(nodes)
                s.nodes[l] = nodes.ctypes.data
                s.nnodes[l] = nodes.shape[0]
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


class Data:
    """Base vectors for verification (FP32) and the walk's storage copy."""

    def __init__(self, base, storage=F32):
        self.base = _f32(base)
        self.storage = storage
        self.walk = self.base if storage == F32 else convert(self.base, storage)
        s = OrcData()
        s.n, s.d = self.base.shape
        s.base = self.base.ctypes.data
        s.walk_storage = storage
        s.walk_base = self.walk.ctypes.data
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


@dataclasses.dataclass
class Params:
    tau: float = 0.92
    cutoff: float = 1.4
    t_param: int = 0
    kappa: int = 0
    w: int = 1
    early_abort: int = 1
    g: int = 8
    v: int = 4
    cache_slots: int = 0
    variant: int = VARIANT_STD  # VARIANT_EXT: g1 = G_0.5 (L0.5), g2 = G_1 (L1), cutoff 0.6 (Sec. 4.5)
    walk_p: float = 0.0  # VARIANT_PGRAPH: g1 = G_p walked under L_walk_p (Sec. 4.3's per-p HNSW)

    def c(self) -> OrcParams:
        return OrcParams(self.tau, self.cutoff, self.t_param, self.kappa, self.w, self.early_abort,
                         self.g, self.v, self.cache_slots, self.variant, self.walk_p)


def knn_search(G: Graph, D: Data, q, metric, ef, t, w=1, g=8, v=4, cache_slots=0, mp=0.0):
    """C (ids, base keys) and stats of KnnSearch for one query (mp: the p of metric LP)."""
    q = _f32(q)
    ids = np.empty(max(t, 1), np.int32)
    keys = np.empty(max(t, 1), np.float32)
    st = OrcStats()
    nc = _load().orc_knn_search(G.ref, D.ref, _ptr(q), metric, float(mp), ef, t, w, g, v, cache_slots,
                                _ptr(ids), _ptr(keys), ctypes.byref(st))
    return ids[:nc], keys[:nc], st


def verify(D: Data, q, p, K, C, kappa, m, early_abort=1):
    """Algorithm 1's verification over candidate list C; returns (ids, S, dist, stats)."""
    q = _f32(q)
    C = np.ascontiguousarray(C, np.int32)
    ids = np.empty(K, np.int32)
    S = np.empty(K, np.float64)
    dist = np.empty(K, np.float64)
    st = OrcStats()
    nr = _load().orc_verify(D.ref, _ptr(q), float(p), K, _ptr(C), C.shape[0], kappa, m, early_abort,
                            _ptr(ids), _ptr(S), _ptr(dist), ctypes.byref(st))
    return ids[:nr], S[:nr], dist[:nr], st


def query_batch(g1: Graph, g2: Graph, D: Data, queries, p, k, ef, prm: Params | None = None,
                k_stride=None, c_stride=0, threads=0):
    """Full query path for each query. Returns dict with ids (int64, -1 pad),
    dist/S (float64, +inf pad), stats (structured), and C ids/keys when
    ``c_stride`` > 0."""
    prm = prm or Params()
    queries = _f32(queries)
    nq = queries.shape[0]
    p = _f32(p)
    k = np.ascontiguousarray(k, np.int32)
    ef = np.ascontiguousarray(ef, np.int32)
    ks = int(k_stride or (k.max() if nq else 1))
    ids = np.empty((nq, ks), np.int64)
    dist = np.empty((nq, ks), np.float64)
    S = np.empty((nq, ks), np.float64)
    stats = np.zeros(nq, STATS_DTYPE)
    cids = ckeys = None
    if c_stride:
        cids = np.full((nq, c_stride), -1, np.int32)
        ckeys = np.full((nq, c_stride), np.inf, np.float32)
    pc = prm.c()
    _load().orc_query_batch(g1.ref, g2.ref, D.ref, _ptr(queries), nq, _ptr(p), _ptr(k), _ptr(ef),
                            ctypes.byref(pc), ks, _ptr(ids), _ptr(dist), _ptr(S), c_stride,
                            _ptr(cids), _ptr(ckeys), _ptr(stats), threads)
    out = dict(ids=ids, dist=dist, S=S, stats=stats)
    if c_stride:
        out["c_ids"] = cids
        out["c_keys"] = ckeys
    return out
