"""The two HNSW base graphs (G1 under L1, G2 under L2; or, for the extended
variant of the U-HNSW paper's Sec. 4.5, G_0.5 under L0.5 and G_1) as
per-layer CSR.

``build_graph`` runs the deterministic C builder in ``hnsw_build.c`` and
returns a :class:`Graph`. Built graphs are cached on disk (keyed by the
workload digest, metric, M, efConstruction, seed and builder version) under
``$UHNSW_CACHE`` (default ``<repo>/_cache``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hnsw_build.c")
_LIB = os.path.join(_HERE, "_hnsw_build.so")
BUILDER_VERSION = "hb2"

_lib = None


def build_lib(force: bool = True) -> str:
    """Compile the builder into ``synth/_hnsw_build.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        lib.hb_build.restype = ctypes.c_void_p
        lib.hb_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int]
        lib.hb_max_level.restype = ctypes.c_int
        lib.hb_max_level.argtypes = [ctypes.c_void_p]
        lib.hb_entry.restype = ctypes.c_int32
        lib.hb_entry.argtypes = [ctypes.c_void_p]
        lib.hb_levels.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.hb_layer_nodes.restype = ctypes.c_int64
        lib.hb_layer_nodes.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.hb_layer_edges.restype = ctypes.c_int64
        lib.hb_layer_edges.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.hb_layer_csr.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.hb_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclasses.dataclass
class Layer:
    nodes: np.ndarray | None  # int32 ascending ids on this layer (None for layer 0 = all)
    row_ptr: np.ndarray       # int64, len(nodes)+1 (n+1 on layer 0)
    col: np.ndarray           # int32 neighbour ids


@dataclasses.dataclass
class Graph:
    metric: int               # 1 -> L1 (G1), 2 -> L2 (G2), 3 -> L0.5 (G_0.5), 4 -> L_p for one p
    n: int
    M: int
    ef_construction: int
    seed: int
    max_level: int
    entry: int
    levels: np.ndarray        # int8 (n,)
    layers: list              # list[Layer], index = layer

    @property
    def M0(self) -> int:
        return 2 * self.M


def _key(wl_digest: str, metric: int, M: int, efc: int, seed: int) -> str:
    s = f"{wl_digest}:{metric}:{M}:{efc}:{seed}:{BUILDER_VERSION}"
    return hashlib.sha256(s.encode()).hexdigest()[:24]


def _cache_dir() -> str:
    d = os.environ.get("UHNSW_CACHE", os.path.join(os.path.dirname(_HERE), "_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def _save(path: str, g: Graph) -> None:
    arrs = {"meta": np.array([g.metric, g.n, g.M, g.ef_construction, g.seed, g.max_level, g.entry],
                             dtype=np.int64),
            "levels": g.levels}
    for l, L in enumerate(g.layers):
        if L.nodes is not None:
            arrs[f"nodes{l}"] = L.nodes
        arrs[f"rp{l}"] = L.row_ptr
        arrs[f"col{l}"] = L.col
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def _load_file(path: str) -> Graph:
    z = np.load(path)
    metric, n, M, efc, seed, ml, ep = (int(x) for x in z["meta"])
    layers = []
    for l in range(ml + 1):
        layers.append(Layer(nodes=z[f"nodes{l}"] if l else None, row_ptr=z[f"rp{l}"], col=z[f"col{l}"]))
    return Graph(metric=metric, n=n, M=M, ef_construction=efc, seed=seed, max_level=ml, entry=ep,
                 levels=z["levels"], layers=layers)


def build_graph(base: np.ndarray, metric: int, M: int = 16, ef_construction: int = 200,
                seed: int = 0, threads: int = 0, cache: bool = True,
                digest: str | None = None, verbose: bool = False, batch_max: int = 1024,
                metric_p: float = 0.0) -> Graph:
    """The HNSW graph of `base` under `metric` (1 L1, 2 L2, 3 L0.5, 4 sum
    |x - y|^metric_p), built by hnsw_build.c in insertion batches of at most
    `batch_max` nodes."""
    base = np.ascontiguousarray(base, dtype=np.float32)
    n, d = base.shape
    path = None
    if cache:
        if digest is None:
            digest = hashlib.sha256(base.tobytes()).hexdigest()
        tag = digest if metric != METRIC_LP else f"{digest}:p{float(metric_p)!r}"
        key = _key(tag, metric, M, ef_construction, seed)
        if batch_max != 1024:
            key = _key(f"{tag}:b{batch_max}", metric, M, ef_construction, seed)
        path = os.path.join(_cache_dir(), f"g_{key}.npz")
        if os.path.exists(path):
            return _load_file(path)
    lib = _load()
    t0 = time.time()
    h = lib.hb_build(base.ctypes.data, n, d, metric, float(metric_p), M, ef_construction, seed, threads,
                     int(verbose), batch_max)
    if not h:
        raise ValueError("hnsw build rejected its arguments")
    try:
        ml = lib.hb_max_level(h)
        ep = lib.hb_entry(h)
        levels = np.empty(n, np.int8)
        lib.hb_levels(h, levels.ctypes.data)
        layers = []
        for l in range(ml + 1):
            nn = lib.hb_layer_nodes(h, l)
            ne = lib.hb_layer_edges(h, l)
            nodes = np.empty(nn, np.int32) if l else None
            rp = np.empty(nn + 1, np.int64)
            col = np.empty(max(ne, 1), np.int32)[:ne]
            lib.hb_layer_csr(h, l, nodes.ctypes.data if l else None, rp.ctypes.data,
                             col.ctypes.data if ne else None)
            layers.append(Layer(nodes=nodes, row_ptr=rp, col=col))
    finally:
        lib.hb_free(h)
    g = Graph(metric=metric, n=n, M=M, ef_construction=ef_construction, seed=seed, max_level=ml,
              entry=ep, levels=levels, layers=layers)
    if verbose:
        print(f"[synth] built G{ {3: '0.5'}.get(metric, metric)} n={n} d={d} in {time.time() - t0:.1f}s",
              flush=True)
    if path is not None:
        _save(path, g)
    return g


METRIC_L1, METRIC_L2, METRIC_L05, METRIC_LP = 1, 2, 3, 4


def build_graphs(wl, threads: int = 0, cache: bool = True, verbose: bool = False, extended: bool = False):
    """(G1, G2) for a :class:`synth.Workload`; with ``extended`` the pair of
    the extended variant, (G_0.5, G_1)."""
    dg = hashlib.sha256(np.ascontiguousarray(wl.base).tobytes()).hexdigest() if cache else None
    metrics = (METRIC_L05, METRIC_L1) if extended else (METRIC_L1, METRIC_L2)
    return tuple(build_graph(wl.base, m, wl.M, wl.ef_construction, wl.graph_seed, threads, cache, dg, verbose)
                 for m in metrics)


def cached_graphs(wl, extended: bool = False):
    """The pair ``build_graphs`` would return, if both are already in the
    cache; else None (nothing is built)."""
    dg = hashlib.sha256(np.ascontiguousarray(wl.base).tobytes()).hexdigest()
    metrics = (METRIC_L05, METRIC_L1) if extended else (METRIC_L1, METRIC_L2)
    paths = [os.path.join(_cache_dir(), f"g_{_key(dg, m, wl.M, wl.ef_construction, wl.graph_seed)}.npz")
             for m in metrics]
    if not all(os.path.exists(p) for p in paths):
        return None
    return tuple(_load_file(p) for p in paths)


def save_fbin(path: str, base: np.ndarray) -> None:
    """Base vectors as .fbin: int32 n, int32 d, then n*d FP32 row-major."""
    base = np.ascontiguousarray(base, np.float32)
    with open(path, "wb") as f:
        f.write(np.array(base.shape, np.int32).tobytes())
        f.write(base.tobytes())


def save_graph_file(path: str, g: Graph) -> None:
    """One graph in the UHG1 layout read by uhnsw_load_graph_files:
    "UHG1", int32 n, M, max_level, entry_point, int8 level[n], then per layer
    int64 n_l, int64 row_ptr[n_l + 1], int32 col[...], and for l >= 1
    int32 nodes[n_l]."""
    n = len(g.levels)
    with open(path, "wb") as f:
        f.write(b"UHG1")
        f.write(np.array([n, g.M, g.max_level, g.entry], np.int32).tobytes())
        f.write(np.ascontiguousarray(g.levels, np.int8).tobytes())
        for l, L in enumerate(g.layers):
            rp = np.ascontiguousarray(L.row_ptr, np.int64)
            f.write(np.array([len(rp) - 1], np.int64).tobytes())
            f.write(rp.tobytes())
            f.write(np.ascontiguousarray(L.col, np.int32).tobytes())
            if l >= 1:
                f.write(np.ascontiguousarray(L.nodes, np.int32).tobytes())
