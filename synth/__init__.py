"""Seeded synthetic inputs for the U-HNSW query path.

This module only draws numbers: base vectors, queries and the per-query
(p, k, ef) tuples of the five workloads, plus (in ``synth.graphs``) the two
HNSW base graphs built over the base vectors. It holds none of the query
path's arithmetic (no candidate walk, no L_p verification). Both the CPU
oracle and the GPU library consume exactly these arrays.

Workload shapes follow the datasets of the U-HNSW paper's evaluation
(Sec. 4.1.1, dataset table: SIFT 128-d, GIST 960-d, GloVe 100-d, Deep-style
96-d), with seeded stand-ins since the datasets themselves are not used.
The query tuple (q, p) and per-query K follow the problem statement
(Sec. 1.1 and Sec. 2.1); p ranges over [0.5, 2] (Sec. 2.1). Workloads 6
and 7 are the inputs of the extended variant (Sec. 4.5): the vectors,
queries and graph seed of workloads 1 and 2, with p over [0.2, 1] instead.

Seeds: workload c uses 1000*c + 1 for base vectors, +2 for queries, +3 for
per-query p/k/ef, +4 for mixture means / per-dimension scales, +5 for the
graph levels (workloads 6 and 7 take those of 1 and 2 except +3, their own).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = ["Workload", "make_workload", "p_uniform", "p_uniform_ext", "P_GRID", "P_GRID_EXT", "WORKLOADS",
           "clustered"]

# p grid 0.5, 0.6, ..., 2.0 (Sec. 4.3 evaluates exactly these 16 values).
P_GRID = np.array([(5 + j) / 10 for j in range(16)], dtype=np.float32)
# the extended variant's range [0.2, 1] on the same 0.1 grid (Sec. 4.5)
P_GRID_EXT = np.array([(2 + j) / 10 for j in range(9)], dtype=np.float32)

WORKLOADS = {
    1: dict(n=10_000, d=32, nq=100, name="gauss-10k-d32"),
    2: dict(n=1_000_000, d=128, nq=10_000, name="mixture-1M-d128"),
    3: dict(n=1_000_000, d=960, nq=1_000, name="gammafeat-1M-d960"),
    4: dict(n=1_183_514, d=100, nq=10_000, name="unitgauss-1.18M-d100"),
    5: dict(n=10_000_000, d=96, nq=2_000, name="unitgauss-10M-d96"),
    6: dict(n=10_000, d=32, nq=100, name="gauss-10k-d32-pext", like=1),
    7: dict(n=1_000_000, d=128, nq=10_000, name="mixture-1M-d128-pext", like=2),
}

_CHUNK = 1 << 17


@dataclasses.dataclass
class Workload:
    cfg: int
    name: str
    base: np.ndarray      # (n, d) float32, row-major
    queries: np.ndarray   # (nq, d) float32
    p: np.ndarray         # (nq,) float32
    k: np.ndarray         # (nq,) int32
    ef: np.ndarray        # (nq,) int32
    graph_seed: int
    M: int = 16
    ef_construction: int = 200

    @property
    def n(self) -> int:
        return int(self.base.shape[0])

    @property
    def d(self) -> int:
        return int(self.base.shape[1])

    @property
    def nq(self) -> int:
        return int(self.queries.shape[0])

    def digest(self) -> str:
        """sha256 over the base vectors, queries and per-query parameters."""
        h = hashlib.sha256()
        for a in (self.base, self.queries, self.p, self.k, self.ef):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def p_uniform(rng: np.random.Generator, size: int) -> np.ndarray:
    """p uniform on (0.5, 2]: p = float32(2 - 1.5 U), U in [0, 1)."""
    u = rng.random(size)
    return (2.0 - 1.5 * u).astype(np.float32)


def p_uniform_ext(rng: np.random.Generator, size: int) -> np.ndarray:
    """p uniform on (0.2, 1]: p = float32(1 - 0.8 U), U in [0, 1)."""
    u = rng.random(size)
    return (1.0 - 0.8 * u).astype(np.float32)


def _gauss(rng, n, d):
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = rng.standard_normal((e - s, d), dtype=np.float32)
    return out


def _unit_gauss(rng, n, d):
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        x = rng.standard_normal((e - s, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = x.astype(np.float32)
    return out


def _mixture(rng_pts, means, n):
    """100-component equal-weight mixture, sigma 32, clipped to [0, 255], rounded."""
    c, d = means.shape
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        comp = rng_pts.integers(0, c, size=e - s)
        x = means[comp] + 32.0 * rng_pts.standard_normal((e - s, d))
        out[s:e] = np.rint(np.clip(x, 0.0, 255.0)).astype(np.float32)
    return out


def _gamma_feat(rng_pts, scales, n):
    """x_ij = |z_ij| * s_j with z ~ N(0, 1) and per-dimension s_j ~ Gamma(2, 0.05)."""
    d = scales.shape[0]
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = rng_pts.standard_normal((e - s, d))
        out[s:e] = (np.abs(z) * scales[None, :]).astype(np.float32)
    return out


def _size_name(n: int) -> str:
    """10_000 -> '10k', 1_183_514 -> '1.18M' (three significant digits)."""
    for div, suf in ((1_000_000, "M"), (1_000, "k")):
        if n >= div:
            return f"{float(f'{n / div:.3g}'):g}{suf}"
    return str(n)


def make_workload(cfg: int, n: int | None = None, nq: int | None = None,
                  d: int | None = None) -> Workload:
    """Build workload ``cfg`` (1..7). ``n``/``nq``/``d`` override the sizes
    (same distribution, same seeds) for reduced test cases."""
    spec = WORKLOADS[cfg]
    n = spec["n"] if n is None else int(n)
    nq = spec["nq"] if nq is None else int(nq)
    d = spec["d"] if d is None else int(d)
    like = spec.get("like", cfg)
    s0 = 1000 * like
    r_base, r_q, r_aux = (_rng(s0 + i) for i in (1, 2, 4))
    r_par = _rng(1000 * cfg + 3)

    if cfg == 6:
        base = _gauss(r_base, n, d)
        queries = _gauss(r_q, nq, d)
        p = p_uniform_ext(r_par, nq)
        k = np.full(nq, 10, np.int32)
        ef = np.full(nq, 128, np.int32)  # p near 0.2 needs a wider walk than workload 1's 64
    elif cfg == 7:
        means = r_aux.uniform(32.0, 224.0, size=(100, d))
        base = _mixture(r_base, means, n)
        queries = _mixture(r_q, means, nq)
        p = P_GRID_EXT[np.arange(nq) % len(P_GRID_EXT)].copy()
        k = np.full(nq, 10, np.int32)
        ef = np.full(nq, 64, np.int32)
    elif cfg == 1:
        base = _gauss(r_base, n, d)
        queries = _gauss(r_q, nq, d)
        p = p_uniform(r_par, nq)
        k = np.full(nq, 10, np.int32)
        ef = np.full(nq, 64, np.int32)
    elif cfg == 2:
        means = r_aux.uniform(32.0, 224.0, size=(100, d))
        base = _mixture(r_base, means, n)
        queries = _mixture(r_q, means, nq)
        p = P_GRID[np.arange(nq) % 16].copy()
        k = np.full(nq, 10, np.int32)
        ef = np.full(nq, 64, np.int32)
    elif cfg == 3:
        scales = r_aux.gamma(2.0, 0.05, size=d)
        base = _gamma_feat(r_base, scales, n)
        queries = _gamma_feat(r_q, scales, nq)
        p = p_uniform(r_par, nq)
        k = np.full(nq, 10, np.int32)
        ef = np.full(nq, 64, np.int32)
    elif cfg == 4:
        base = _unit_gauss(r_base, n, d)
        queries = _unit_gauss(r_q, nq, d)
        p = p_uniform(r_par, nq)
        k = np.array([1, 10, 100], np.int32)[np.arange(nq) % 3]
        ef = np.array([r_par.integers(int(kk), 513) for kk in k], np.int32)
    elif cfg == 5:
        base = _unit_gauss(r_base, n, d)
        queries = _unit_gauss(r_q, nq, d)
        p = p_uniform(r_par, nq)
        k = np.where(r_par.random(nq) < 0.5, 10, 100).astype(np.int32)
        ef = np.maximum(k, 128).astype(np.int32)
    else:
        raise ValueError(f"unknown workload {cfg}")
    name = spec["name"]
    if (n, d) != (spec["n"], spec["d"]):  # reduced case: name its own sizes
        name = f"{name.split('-')[0]}-{_size_name(n)}-d{d}"
    return Workload(cfg=cfg, name=name, base=base, queries=queries,
                    p=p, k=k, ef=ef, graph_seed=s0 + 5)


def clustered(n: int, nq: int, d: int, clusters: int, seed: int, spread: float = 0.05):
    """Tight, well-separated clusters: centres N(0, 1) per coordinate, points
    and queries centre + N(0, spread^2); queries near the first centres, in
    turn. A search list wider than a cluster then holds members of other
    clusters whose distances are many times the near ones'. Returns (base,
    queries) as float32."""
    rng = _rng(seed)
    centres = rng.standard_normal((clusters, d))
    base = centres[np.arange(n) % clusters] + spread * rng.standard_normal((n, d))
    queries = centres[np.arange(nq) % clusters] + spread * rng.standard_normal((nq, d))
    return base.astype(np.float32), queries.astype(np.float32)
