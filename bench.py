#!/usr/bin/env python3
"""Benchmark of the U-HNSW query path on one MI355X.

Workload (the configuration the headline metric is quoted on): n = 1,000,000
base vectors, d = 128, a seeded 100-component Gaussian mixture clipped to
[0, 255] and rounded (SIFT-like); 10,000 queries from the same mixture with
p cycling over {0.5, 0.6, ..., 2.0}; K = 10; HNSW graphs G1 / G2 with M = 16,
efConstruction = 200. Inputs are resident in HBM before the timed region.

A step is one search of all 10,000 queries: candidate walk + L_p
verification (Algorithm 1 of the U-HNSW paper). efSearch is the smallest of
{32, 64, 128, 256} whose recall@10 (against the FP64 brute-force ground
truth on a 2,000-query sample) reaches 0.9; it is chosen before timing.

Prints one JSON line. ``value`` is the plain FP32 form's QPS; the
BF16-storage batched form and the same batching on FP32 rows are reported
beside it in ``forms``.

Other legs: ``--workload 3 | 4 | 5`` (precision, batching and serving forms
on their own inputs), ``--workload 7`` (the same vectors and queries on the
extended index of the paper's Sec. 4.5, p over 0.2..1.0, efSearch from
{128, 256, 384, 512}) and ``--sweep`` (method diagnostics).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

# Two batches in flight need their streams on different hardware queues; HIP
# gives a process four by default and the library and torch hold some.
# Must be set before HIP initialises.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# v_exp_f32 / v_log_f32 issue at half the FP32 rate on gfx950: 256 CUs x 4
# SIMDs x 16 lanes / 2 per cycle at 2.4 GHz (lane operations per second)
TRANS_PEAK = 256 * 4 * 16 / 2 * 2.4e9
# HBM traffic of the walk kernel from two rocprofv3 counter passes
# (profiles/walk_kernel_mixture-1M-d128_ef256_hbm-traffic.md): FETCH_SIZE x 2.0
# + WRITE_SIZE x 1.0 per launch, valid only for that kernel source, the host
# code that plans its launch (cache size, block shape) and ef.
TRAFFIC = {"kernel_sha256_prefix": "4e0681caf673a0af", "host_sha256_prefix": "2a943e38f694996f", "ef": 256,
           "bytes_per_launch": 22.081e9}
# the sources the kernels are compiled from (hashed to tie the counter traffic
# to the code it was measured on)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2605_02030_amd", "csrc", f)
               for f in ("uhnsw_device.h", "uhnsw_walk_part.hip", "uhnsw_kernels.hip", "uhnsw_internal.h")]
HOST_SRC = os.path.join(ROOT, "paper_2605_02030_amd", "csrc", "uhnsw_host.cpp")
GT_PATH = os.path.join(ROOT, "tests", "golden", "gt_mixture-1M-d128.npz")
EF_GRID = (32, 64, 128, 256)
# the extended index's p near 0.2 needs a wider walk (oracle recall@10 at
# ef 256 / 512: 0.89 / 0.95 on workload 7)
EF_GRID_EXT = (128, 256, 384, 512)
# --reduced: the serving form's workload at 1M rows (graphs from the CPU
# builder's cache); by default it runs at its 10M rows with graphs built on
# the GPU
REDUCED_N = {5: 1_000_000}
# efSearch grid of the secondary workloads' sweeps: through EFMAX, to state
# the recall each input can reach
EF_SWEEP = (32, 64, 128, 256, 512, 1024, 2048)
TARGET_RECALL = 0.9


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def recall_at_k(ids, gt_ids, qidx, K=10):
    got = ids[qidx, :K]
    return float(np.mean([len(set(got[i].tolist()) & set(gt_ids[i].tolist())) / K for i in range(len(qidx))]))


class Form:
    """One configured search path on the resident index."""

    def __init__(self, torch, uhnsw, wl, g1, g2, storage, persistent, name, variant=0):
        self.torch, self.uhnsw, self.name = torch, uhnsw, name
        self.ctx = uhnsw.Context(0)
        t0 = time.time()
        self.ctx.load_graphs(wl.base, g1, g2, storage=storage, variant=variant)
        log(f"{name}: index uploaded in {time.time() - t0:.1f}s")
        self.persistent = persistent
        dev = torch.device("cuda:0")
        self.nq = wl.nq
        self.q = torch.from_numpy(wl.queries).to(dev)
        self.p = torch.from_numpy(wl.p).to(dev)
        self.k = torch.from_numpy(wl.k).to(dev)
        # the batching form pipelines consecutive steps on two streams (each
        # with its own outputs) so one step's tail overlaps the next one's head
        self.pipeline = 2 if persistent else 1
        self.streams = [torch.cuda.Stream() for _ in range(self.pipeline)] if self.pipeline > 1 else [None]
        self.outs = [(torch.empty((wl.nq, 10), dtype=torch.int64, device=dev),
                      torch.empty((wl.nq, 10), dtype=torch.float32, device=dev),
                      torch.zeros((wl.nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev))
                     for _ in range(self.pipeline)]
        self.n_steps = 0
        self.ef_val = None
        self.ef = None
        self.tuned = {}

    def set_ef(self, ef, knobs=None):
        """knobs (batched forms): fixed beam_width / visited_slots /
        waves_per_block / persistent / waves_per_cu instead of the autotuner's
        choice, e.g. to profile one configuration without the tuning launches."""
        self.ef_val = ef
        self.ef = self.torch.full((self.nq,), ef, dtype=torch_int32(self.torch), device="cuda:0")
        if self.persistent and knobs and ef not in self.tuned:
            t = self.uhnsw.default_params(fused=1, graph=1, **knobs)
            self.tuned[ef] = t
            log(f"{self.name} ef={ef}: fixed knobs {knobs}")
        if self.persistent and ef not in self.tuned:
            base = self.uhnsw.default_params(fused=1, persistent=1, graph=1)
            t = self.ctx.autotune(self.q, self.p, self.k, self.ef, 10, ef, params=base, allow_beam=True,
                                  pipelined=self.pipeline > 1, stream=self.streams[0])
            t.graph = 1
            self.tuned[ef] = t
            log(f"{self.name} ef={ef}: autotuned beam={t.beam_width} slots={t.visited_slots} "
                f"wpb={t.waves_per_block} persistent={t.persistent}")

    def step(self, timing=False, graph=True):
        if self.persistent:  # batching form: fused persistent launch, autotuned, replayed as a hipGraph
            prm = self.uhnsw.uhnsw_params.from_buffer_copy(self.tuned[self.ef_val])
            prm.timing = int(timing)
            prm.graph = int(graph)
        else:
            prm = self.uhnsw.default_params(timing=int(timing))
        j = self.n_steps % self.pipeline
        ids, dists, stats = self.outs[j]
        self.ctx.search_device(self.q, self.p, self.k, self.ef, 10, self.ef_val, ids, dists, stats, params=prm,
                               stream=self.streams[j])
        self.n_steps += 1

    @property
    def ids(self):  # outputs of the last step
        return self.outs[(self.n_steps - 1) % self.pipeline][0]

    def stats_np(self):
        st = self.outs[(self.n_steps - 1) % self.pipeline][2]
        return st.cpu().numpy().view(self.uhnsw.STATS_DTYPE).reshape(self.nq)


def torch_int32(torch):
    return torch.int32


def host_api_qps(form, wl, ef, uhnsw, calls=5):
    """uhnsw_search (host arrays in and out, copies over PCIe inside the
    call, launch sequence replayed as one hipGraph): queries per second of
    wall time per call. Reported beside ``value``, never as it."""
    efa = np.full(wl.nq, ef, np.int32)
    prm = uhnsw.default_params(graph=1)
    for _ in range(2):
        form.ctx.search(wl.queries, wl.p, wl.k, efa, params=prm)
    t0 = time.perf_counter()
    for _ in range(calls):
        form.ctx.search(wl.queries, wl.p, wl.k, efa, params=prm)
    return round(wl.nq * calls / (time.perf_counter() - t0), 1)


def calibrate(form, gt, log_prefix, grid=EF_GRID):
    torch = form.torch
    chosen, table = None, []
    for ef in grid:
        form.set_ef(ef)
        form.step()
        form.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        form.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = recall_at_k(form.ids.cpu().numpy(), gt["ids"], gt["qidx"])
        table.append({"ef": ef, "recall@10": round(rec, 4), "qps_probe": round(form.nq / dt, 1)})
        log(f"{log_prefix} ef={ef}: recall@10={rec:.4f}  probe {form.nq / dt:,.0f} QPS")
        if rec >= TARGET_RECALL and chosen is None:
            chosen = ef
            break
    if chosen is None:  # report the best reachable point honestly
        chosen = max(table, key=lambda r: r["recall@10"])["ef"]
    form.set_ef(chosen)
    return chosen, table


def timed(form, steps, warmup, wl, rate_khz):
    """Time `steps` steps after `warmup`. Kernel times come from HIP events on
    the launch stream: the pre-pass, the walk (or fused) kernel and the
    verification kernel separately (the batched forms: from one uncaptured
    launch with the same knobs after the timed region)."""
    torch = form.torch
    for _ in range(warmup):
        form.step()
    torch.cuda.synchronize()
    split = []
    t0 = time.perf_counter()
    for _ in range(steps):
        if form.pipeline > 1:  # steps overlap: no per-step wait
            form.step()
            continue
        form.step(timing=True)
        split.append(form.ctx.last_timing_split())  # waits for this step's events
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    if form.pipeline > 1:  # one launch's own kernels, measured alone after the timed region (5 launches)
        for _ in range(5):
            form.step(timing=True, graph=False)
            split.append(form.ctx.last_timing_split())
    pre, walk, ver = (float(np.mean([x[i] for x in split])) for i in range(3))
    walks = np.array([x[1] for x in split])
    st = form.stats_np()
    t0c = st["t_begin"].astype(np.int64)
    t1c = st["t_end"].astype(np.int64)
    start = t0c.min()
    lat_ms = ((t1c - start) % (1 << 32)) / rate_khz  # ticks -> ms
    return dict(total_s=total, prepass_ms=pre, walk_ms=walk, verify_ms=ver,
                walk_reps=len(walks), walk_ms_median=float(np.median(walks)),
                walk_ms_range=[float(walks.min()), float(walks.max())],
                p50_ms=float(np.percentile(lat_ms, 50)), p99_ms=float(np.percentile(lat_ms, 99)), stats=st,
                n_b=float(st["n_b"].mean()), n_exp=float(st["n_exp"].mean()), n_p=float(st["n_p"].mean()),
                flags=int((st["flags"] != 0).sum()))


def method_bytes(wl, elem, gpu_st, counts, fused):
    """Bytes the method itself reads in one launch of the walk (or fused)
    kernel: the layer-0 rows N_b - N_up of d x elem bytes and the N_exp
    adjacency rows of 2M = 32 ids (128 B) per query, with N_b and N_exp from
    the oracle's walk over an exact visited set (the descent's N_up rows are
    the pre-pass kernel's, and identical on both sides); the fused kernel
    also reads the N_p FP32 rows it verifies. Returns (walk-kernel bytes,
    pre-pass bytes)."""
    up = gpu_st["n_up"].astype(np.float64).sum()
    l0 = counts["n_b"].astype(np.float64).sum() - up
    walk = l0 * wl.d * elem + counts["n_exp"].astype(np.float64).sum() * 32 * 4
    if fused:
        walk += gpu_st["n_p"].astype(np.float64).sum() * wl.d * 4
    return float(walk), float(up * wl.d * elem)


def serving(torch, uhnsw, wl, g1, g2, gt, ef, rates=(20_000, 50_000, 100_000, 200_000), seconds=5.0,
            warmup_s=0.5, storage=None, k=None, k_max=10, label="BF16", variant=0, params=None):
    """Serving form: Poisson arrivals into the continuous-batching server.
    Arrival i carries query i mod nq. Each offered rate runs `warmup_s` of
    arrivals that are not counted, then `seconds` of measured arrivals:
    achieved QPS over the measured arrivals' span, their p50 / p99 / p99.9
    latency (completion minus scheduled arrival, queueing included). `k`
    gives each query's K (default: the workload's), `ef` one efSearch for
    all; admission slots follow the fused kernel's LDS plan."""
    ctx = uhnsw.Context(0)
    ctx.load_graphs(wl.base, g1, g2, storage=uhnsw.STORE_BF16 if storage is None else storage, variant=variant)
    kq = wl.k if k is None else k
    prm = params or uhnsw.default_params(beam_width=2, visited_slots=1024)
    out = []
    gt_row = np.full(wl.nq, -1, np.int64)
    gt_row[gt["qidx"]] = np.arange(len(gt["qidx"]))
    for rate in rates:
        n = int(rate * (seconds + warmup_s))
        qi = (np.arange(n) % wl.nq).astype(np.int32)
        rng = np.random.Generator(np.random.PCG64(rate))
        arrival = np.cumsum(rng.exponential(1e6 / rate, n))
        srv = uhnsw.Server(ctx, k_max=k_max, ef_max=ef, params=prm)
        try:
            ids, dists, status, t_sub, t_launch, t_done = srv.drive(wl.queries, wl.p[qi], kq[qi],
                                                                    np.full(n, ef, np.int32), arrival, out_k=10,
                                                                    qidx=qi)
            info = srv.info()
        finally:
            srv.stop()
        meas = arrival >= warmup_s * 1e6
        lat_ms = (t_done - t_sub)[meas] / 1e3
        span_s = (t_done[meas].max() - arrival[meas][0]) / 1e6
        sel = np.flatnonzero(meas & (gt_row[qi] >= 0))
        rec = float(np.mean([len(set(ids[i, :10].tolist()) & set(gt["ids"][gt_row[qi[i]]].tolist())) / 10
                             for i in sel[:20000]])) if len(sel) else None
        r = dict(offered_qps=rate, measured_queries=int(meas.sum()), measured_s=round(float(span_s), 3),
                 warmup_queries=int((~meas).sum()), achieved_qps=round(float(meas.sum() / span_s), 1),
                 p50_ms=round(float(np.percentile(lat_ms, 50)), 3), p99_ms=round(float(np.percentile(lat_ms, 99)), 3),
                 p999_ms=round(float(np.percentile(lat_ms, 99.9)), 3), mean_ms=round(float(lat_ms.mean()), 3),
                 recall_at_10=round(rec, 4) if rec is not None else None, batches=info["batches"],
                 max_batches_in_flight=info["max_overlap"], slots=info["slots"],
                 waves_per_cu=info["waves_per_cu"], errors=int((status != 0).sum()))
        log("serving", json.dumps(r))
        out.append(r)
    ctx.close()
    return dict(form=f"{label} walk, beam {prm.beam_width}, fused launches on 2 streams, continuous batching",
                ef=ef, k=sorted(set(int(x) for x in np.unique(kq))), rates=out)


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:  # lscpu missing: fall back to /proc
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, g1, g2, ef, variant=0, combos=(), runs=5):
    """The oracle (plain C, OpenMP over queries) timed on the host cores, and
    the method's own work per query from the same runs.

    Timed: all queries of the workload at `ef` with the paper's beam width 1
    and FP32 rows, the median of `runs` runs after one warm-up, on
    OMP_NUM_THREADS threads (the host's CPU share; every core when unset),
    plus one single-thread run over the first 500 queries.

    Method counts: for each (ef, beam width, storage) a GPU form ran with,
    the oracle's N_b and N_exp per query, from its walk over an exact visited
    set: the rows the method reads, without the re-reads the GPU's bounded
    visited cache causes. These are the algorithmic bytes of the roofline."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    G1, G2 = oracle.Graph(g1), oracle.Graph(g2)
    efa = np.full(wl.nq, ef, np.int32)

    def prm(w=1):
        return oracle.Params(variant=variant, cutoff=0.6 if variant else 1.4, w=w)

    D32 = oracle.Data(wl.base)
    oracle.query_batch(G1, G2, D32, wl.queries, wl.p, wl.k, efa, prm(), threads=threads)  # warm-up
    times, out = [], None
    for _ in range(runs):
        t0 = time.perf_counter()
        out = oracle.query_batch(G1, G2, D32, wl.queries, wl.p, wl.k, efa, prm(), threads=threads)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    n1 = min(500, wl.nq)
    t0 = time.perf_counter()
    oracle.query_batch(G1, G2, D32, wl.queries[:n1], wl.p[:n1], wl.k[:n1], efa[:n1], prm(), threads=1)
    dt1 = time.perf_counter() - t0
    counts = {(ef, 1, 0): out["stats"]}
    storages = {0: D32}
    for e, w, storage in sorted(set(combos)):
        if (e, w, storage) in counts:
            continue
        if storage not in storages:
            storages[storage] = oracle.Data(wl.base, storage=storage)
        counts[(e, w, storage)] = oracle.query_batch(G1, G2, storages[storage], wl.queries, wl.p, wl.k,
                                                     np.full(wl.nq, e, np.int32), prm(w), threads=threads)["stats"]
    base = dict(value=round(wl.nq / dt, 1), unit="queries/s", cores=threads, kind="oracle",
                sample=f"all {wl.nq} queries at ef={ef}, beam 1, FP32 rows, same graphs and parameters; "
                       f"median of {runs} runs ({', '.join(f'{t:.2f}' for t in times)} s)",
                single_core_qps=round(n1 / dt1, 1), single_core_sample=f"first {n1} queries, 1 thread",
                nproc=os.cpu_count(), affinity_cpus=len(os.sched_getaffinity(0)), cpu_model=_cpu_model())
    return base, counts


def gt_for(wl):
    path = os.path.join(ROOT, "tests", "golden", f"gt_{wl.name}.npz")
    gt = dict(np.load(path))
    if bytes(gt["digest"]).decode() != wl.digest():
        raise SystemExit(f"{path} does not match the generated workload")
    return gt


def lp_dist64(base, q, ids, p):
    x = base[ids].astype(np.float64)
    return (np.abs(x - q.astype(np.float64)) ** float(p)).sum(1) ** (1.0 / float(p))


def run_secondary(a, torch, uhnsw, sg, synth):
    """Workload 3 (precision form), 4 (batching form) or 5 (serving form, at
    a tenth of its size): one JSON line."""
    t0 = time.time()
    wl = synth.make_workload(a.workload, n=REDUCED_N.get(a.workload) if a.reduced else None)
    log(f"workload {wl.name}: n={wl.n} d={wl.d} nq={wl.nq} ({time.time() - t0:.1f}s)")
    gt = gt_for(wl)
    out = {"workload": wl.name, "n": wl.n, "d": wl.d, "queries": wl.nq, "forms": {}}
    cached = sg.cached_graphs(wl)
    if cached is None:  # not built on the CPU: construct G1 and G2 on the GPU (the same graphs, edge for edge)
        bctx = uhnsw.Context(0)
        graphs = []
        for metric in (sg.METRIC_L1, sg.METRIC_L2):
            g = uhnsw.build_graph(bctx, wl.base, metric, M=wl.M, ef_construction=wl.ef_construction,
                                  seed=wl.graph_seed)
            log(f"GPU build metric {metric}: {g.seconds:.1f}s, {g.batches} batches, max level {g.max_level}")
            graphs.append(g)
        bctx.close()
        g1, g2 = graphs
        out["graph_build"] = {"where": "GPU (uhnsw_build_graph)", "M": wl.M,
                              "efConstruction": wl.ef_construction,
                              "seconds": {"G1": round(g1.seconds, 1), "G2": round(g2.seconds, 1)},
                              "batches": g1.batches}
    else:
        g1, g2 = cached
    dev = torch.device("cuda:0")
    q = torch.from_numpy(wl.queries).to(dev)
    p = torch.from_numpy(wl.p).to(dev)
    k = torch.from_numpy(wl.k).to(dev)
    kmax = int(wl.k.max())
    ids = torch.empty((wl.nq, kmax), dtype=torch.int64, device=dev)
    dists = torch.empty((wl.nq, kmax), dtype=torch.float32, device=dev)
    stats = torch.zeros((wl.nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev)

    spare = (torch.empty_like(ids), torch.empty_like(dists), torch.empty_like(stats))
    streams = (torch.cuda.Stream(), torch.cuda.Stream())

    def timed_run(ctx, ef_t, efmax, prm, steps, pipeline=1):
        """Seconds per launch; with pipeline=2 consecutive launches alternate
        between two streams and output sets (the last one lands in ids)."""
        sets = ((ids, dists, stats), spare)
        for i in range(2):
            o = sets[i % pipeline]
            ctx.search_device(q, p, k, ef_t, kmax, efmax, *o, params=prm, stream=streams[i % pipeline])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            j = (i + 1 - steps) % pipeline  # the last launch uses the first set
            ctx.search_device(q, p, k, ef_t, kmax, efmax, *sets[j], params=prm, stream=streams[j])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def quality(ids_np, dists_np):
        got = ids_np[gt["qidx"], :10]
        rec = float(np.mean([len(set(got[i].tolist()) & set(gt["ids"][i].tolist())) / 10
                             for i in range(len(got))]))
        err = 0.0
        for i in gt["qidx"][:50]:
            kk = int(wl.k[i])
            sel = ids_np[i, :kk]
            d64 = lp_dist64(wl.base, wl.queries[i], sel, wl.p[i])
            err = max(err, float(np.max(np.abs(dists_np[i, :kk] - d64) / d64)))
        return rec, err

    def sweep_ef(ctx, prm_kw, label, grid=EF_SWEEP):
        """ef_i = max(k_i, E) over the grid (stops after the first E reaching
        the target recall): QPS of one launch of all queries, recall@10."""
        rows = []
        for E in grid:
            ef_np = np.maximum(wl.k, E).astype(np.int32)
            ef_t = torch.from_numpy(ef_np).to(dev)
            dt = timed_run(ctx, ef_t, int(ef_np.max()), uhnsw.default_params(**prm_kw), max(3, a.steps // 4))
            rec, err = quality(ids.cpu().numpy(), dists.cpu().numpy())
            st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(wl.nq)
            rows.append(dict(E=E, qps=round(wl.nq / dt, 1), recall_at_10=round(rec, 4), max_rel_dist_err=err,
                             mean_n_b=round(float(st["n_b"].mean()), 1)))
            log(label, json.dumps(rows[-1]))
            if rec >= TARGET_RECALL:
                break
        return rows

    if a.workload == 5:
        ctx = uhnsw.Context(0)
        ctx.load_graphs(wl.base, g1, g2, storage=uhnsw.STORE_F16)
        # recall reachable through EFMAX (ef_i = max(k_i, E)), FP16 walk, FP32 re-rank
        sweep = sweep_ef(ctx, dict(fused=1), "fp16 sweep")
        ok = [r for r in sweep if r["recall_at_10"] >= TARGET_RECALL]
        pick = ok[0] if ok else max(sweep, key=lambda r: r["recall_at_10"])
        out["ef_sweep"] = sweep
        # the batching form at the chosen E: autotuned, one persistent launch, hipGraph
        ef_np = np.maximum(wl.k, pick["E"]).astype(np.int32)
        ef_t = torch.from_numpy(ef_np).to(dev)
        efmax = int(ef_np.max())
        prm = ctx.autotune(q, p, k, ef_t, kmax, efmax, params=uhnsw.default_params(fused=1, persistent=1),
                           allow_beam=True)
        prm.graph = 1
        dt = timed_run(ctx, ef_t, efmax, prm, a.steps)
        rec, err = quality(ids.cpu().numpy(), dists.cpu().numpy())
        out["forms"]["fp16-batched"] = dict(E=pick["E"], qps=round(wl.nq / dt, 1), ms_per_launch=round(dt * 1e3, 3),
                                            recall_at_10=round(rec, 4), max_rel_dist_err=err,
                                            beam=prm.beam_width, slots=prm.visited_slots,
                                            wpb=prm.waves_per_block, persistent=prm.persistent)
        log("fp16-batched", json.dumps(out["forms"]["fp16-batched"]))
        ctx.close()
        # serving: at the configuration's own ef (max(k, 128)) and at the chosen E
        out["serving"] = []
        for E in sorted({128, pick["E"]}):
            out["serving"].append(serving(torch, uhnsw, wl, g1, g2, gt, max(E, kmax), storage=uhnsw.STORE_F16,
                                          k_max=kmax, label=f"FP16 (E={E})",
                                          params=uhnsw.default_params(beam_width=1)))
    elif a.workload == 4:
        ctx = uhnsw.Context(0)
        ctx.load_graphs(wl.base, g1, g2)
        out["ef_sweep"] = sweep_ef(ctx, {}, "sweep (ef_i = max(k_i, E))")
        ctx.close()
        ef_t = torch.from_numpy(wl.ef).to(dev)
        efmax = int(wl.ef.max())
        for name, batched, pipe in (("plain", False, 1), ("batched", True, 1), ("batched-2-streams", True, 2)):
            ctx = uhnsw.Context(0)
            ctx.load_graphs(wl.base, g1, g2)
            if batched:
                prm = ctx.autotune(q, p, k, ef_t, kmax, efmax,
                                   params=uhnsw.default_params(fused=1, persistent=1), allow_beam=True,
                                   pipelined=pipe > 1, stream=streams[0])
                prm.graph = 1
                knobs = dict(beam=prm.beam_width, slots=prm.visited_slots, wpb=prm.waves_per_block,
                             persistent=prm.persistent)
            else:
                prm = uhnsw.default_params()
                knobs = {}
            dt = timed_run(ctx, ef_t, efmax, prm, a.steps, pipeline=pipe)
            rec, err = quality(ids.cpu().numpy(), dists.cpu().numpy())
            st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(wl.nq)
            lat = ((st["t_end"].astype(np.int64) - st["t_begin"].astype(np.int64).min()) % (1 << 32)) / \
                ctx.device_info()[1]
            out["forms"][name] = dict(qps=round(wl.nq / dt, 1), ms_per_launch=round(dt * 1e3, 3),
                                      recall_at_10=round(rec, 4), max_rel_dist_err=err,
                                      p50_ms=round(float(np.percentile(lat, 50)), 3),
                                      p99_ms=round(float(np.percentile(lat, 99)), 3), **knobs)
            log(name, json.dumps(out["forms"][name]))
            ctx.close()
    else:
        for name, storage in (("fp32", uhnsw.STORE_F32), ("bf16", uhnsw.STORE_BF16), ("fp16", uhnsw.STORE_F16)):
            ctx = uhnsw.Context(0)
            ctx.load_graphs(wl.base, g1, g2, storage=storage)
            sweep = []
            for ef in EF_SWEEP:
                ef_t = torch.full((wl.nq,), ef, dtype=torch.int32, device=dev)
                prm = uhnsw.default_params(fused=1)
                dt = timed_run(ctx, ef_t, ef, prm, a.steps)
                rec, err = quality(ids.cpu().numpy(), dists.cpu().numpy())
                sweep.append(dict(ef=ef, qps=round(wl.nq / dt, 1), recall_at_10=round(rec, 4),
                                  max_rel_dist_err=err))
                log(name, json.dumps(sweep[-1]))
            ok = [s for s in sweep if s["recall_at_10"] >= TARGET_RECALL]
            best = max(ok, key=lambda s: s["qps"]) if ok else max(sweep, key=lambda s: s["recall_at_10"])
            out["forms"][name] = dict(best=best, sweep=sweep)
            ctx.close()
    print(json.dumps(out), flush=True)


SWEEP_GT_PATH = os.path.join(ROOT, "tests", "golden", "gt_sweep_mixture-1M-d128.npz")


def run_sweep(a, torch, uhnsw, sg, synth):
    """Diagnostics of the method on the headline workload (plain FP32 path,
    whole 10,000-query launches, recall on the 200-query sample of the sweep
    ground truth):
      ablation: the verification ablation of Sec. 4.4 (Table 2) at p = 0.51
          and 0.9 -- recall of the first K of C (base-metric order) vs after
          verification, walk and verification time per launch, and the
          verification time with early stop off (tau > 1: all t candidates);
      t_tau: the parameter study of Sec. 4.4 (Fig. 5): t in 100..500 at the
          default tau, tau in 0.75..0.95 at t = 300; ef = 500, K = 50, p
          spread over the 0.1 grid;
      cutoff: recall at each p with the walk forced onto G1 or G2 (the
          crossover the graph-choice cutoff of Sec. 3.1 rests on);
      per_p_hnsw: at p = 0.5, 0.7, 1.2 and 1.8, U-HNSW (G1 / G2 +
          verification) against HNSW on a graph built for that p (built on
          the GPU under sum |x - q|^p and walked under it), efSearch swept
          to the first reaching recall@10 0.9 (Sec. 4.3, Fig. 4).
    One JSON line."""
    wl = synth.make_workload(2)
    gt = dict(np.load(SWEEP_GT_PATH))
    if bytes(gt["digest"]).decode() != wl.digest():
        raise SystemExit(f"{SWEEP_GT_PATH} does not match the generated workload")
    g1, g2 = sg.build_graphs(wl, cache=True, verbose=True)
    ctx = uhnsw.Context(0)
    ctx.load_graphs(wl.base, g1, g2)
    dev = torch.device("cuda:0")
    nq = wl.nq
    qidx, grid, gt_ids = gt["qidx"], gt["p"], gt["ids"]
    grid16 = [float(v) for v in grid if abs(float(v) - 0.51) > 1e-6]
    KM, EFM = 50, 512
    q = torch.from_numpy(wl.queries).to(dev)
    ids = torch.empty((nq, KM), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, KM), dtype=torch.float32, device=dev)
    stats = torch.zeros((nq, uhnsw.STATS_WORDS), dtype=torch.int32, device=dev)
    cid = torch.empty((nq, EFM), dtype=torch.int32, device=dev)
    ckey = torch.empty((nq, EFM), dtype=torch.float32, device=dev)

    def gt_row(pv, s):
        j = int(np.argmin(np.abs(grid - np.float32(pv))))
        assert abs(float(grid[j]) - float(pv)) < 1e-6
        return gt_ids[j, s]

    def run(p_all, K, ef, steps=10, ctx=ctx, **kw):
        tp = torch.from_numpy(np.ascontiguousarray(p_all, np.float32)).to(dev)
        tk = torch.full((nq,), K, dtype=torch.int32, device=dev)
        te = torch.full((nq,), ef, dtype=torch.int32, device=dev)
        prm = uhnsw.default_params(**kw)
        ctx.search_device(q, tp, tk, te, K, ef, ids, dists, stats, cid, ckey, params=prm)
        torch.cuda.synchronize()
        got, cand = ids.cpu().numpy(), cid.cpu().numpy()
        st = stats.cpu().numpy().view(uhnsw.STATS_DTYPE).reshape(nq)
        rec = rec_c = 0.0
        for s, i in enumerate(qidx):
            want = set(gt_row(p_all[i], s)[:K].tolist())
            rec += len(want & set(got[i, :K].tolist())) / K
            rec_c += len(want & set(cand[i, :K].tolist())) / K
        for _ in range(2):
            ctx.search_device(q, tp, tk, te, K, ef, ids, dists, stats, params=prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.search_device(q, tp, tk, te, K, ef, ids, dists, stats, params=prm)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        prm.timing = 1
        ctx.search_device(q, tp, tk, te, K, ef, ids, dists, stats, params=prm)
        w, v = ctx.last_timing()
        return dict(recall=round(rec / len(qidx), 4), recall_first_k_of_c=round(rec_c / len(qidx), 4),
                    qps=round(nq / dt, 1), walk_ms=round(w, 4), verify_ms=round(v, 4),
                    mean_n_p=round(float(st["n_p"].mean()), 2), mean_n_b=round(float(st["n_b"].mean()), 1))

    out = {"workload": wl.name, "n": wl.n, "d": wl.d, "queries_per_launch": nq, "recall_sample": len(qidx),
           "ablation": [], "t_tau": {"t": [], "tau": []}, "cutoff": []}
    for K, ef in ((50, 500), (10, 256)):
        for pv in (0.51, 0.9):
            p_all = np.full(nq, pv, np.float32)
            r = run(p_all, K, ef)
            r_ns = run(p_all, K, ef, tau=1.01)
            row = dict(K=K, ef=ef, t=min(ef, 6 * K), p=pv, recall_after_filtering=r["recall_first_k_of_c"],
                       recall_after_reranking=r["recall"], generation_ms=r["walk_ms"],
                       verification_ms=r["verify_ms"], verification_no_early_stop_ms=r_ns["verify_ms"],
                       mean_n_p=r["mean_n_p"], mean_n_p_no_early_stop=r_ns["mean_n_p"], qps=r["qps"],
                       qps_no_early_stop=r_ns["qps"])
            out["ablation"].append(row)
            log("ablation", json.dumps(row))
    p_mix = wl.p.copy()
    for s, i in enumerate(qidx):
        p_mix[i] = grid16[s % len(grid16)]
    for t in (100, 200, 300, 400, 500):
        r = run(p_mix, 50, 500, t=t)
        out["t_tau"]["t"].append(dict(t=t, tau=0.92, recall_at_50=r["recall"], qps=r["qps"],
                                      mean_n_p=r["mean_n_p"]))
        log("t", json.dumps(out["t_tau"]["t"][-1]))
    for tau in (0.75, 0.80, 0.85, 0.90, 0.92, 0.95):
        r = run(p_mix, 50, 500, tau=tau)
        out["t_tau"]["tau"].append(dict(t=300, tau=tau, recall_at_50=r["recall"], qps=r["qps"],
                                        mean_n_p=r["mean_n_p"]))
        log("tau", json.dumps(out["t_tau"]["tau"][-1]))
    for pv in [float(v) for v in grid]:
        p_all = np.full(nq, pv, np.float32)
        row = {"p": round(pv, 2)}
        for name, cutoff in (("G1", 10.0), ("G2", 0.01), ("default", 1.4)):
            r = run(p_all, 10, 256, steps=3, cutoff=cutoff)
            row[name] = dict(recall_at_10=r["recall"], qps=r["qps"])
        out["cutoff"].append(row)
        log("cutoff", json.dumps(row))
    # Sec. 4.3, Fig. 4: U-HNSW against HNSW on a graph built for the query's
    # own p (GPU build under sum |x - q|^p, walked under the same key), at
    # four p; the first efSearch of each that reaches recall@10 0.9
    out["per_p_hnsw"] = {"rows": [], "summary": []}
    efs = (32, 64, 128, 192, 256, 384, 512)
    for pv in (0.5, 0.7, 1.2, 1.8):
        p_all = np.full(nq, pv, np.float32)
        bctx = uhnsw.Context(0)
        gp = uhnsw.build_graph(bctx, wl.base, uhnsw.METRIC_LP, M=wl.M, ef_construction=wl.ef_construction,
                               seed=wl.graph_seed, metric_p=pv)
        bctx.close()
        log(f"per-p: G_{pv} built on the GPU in {gp.seconds:.1f}s")
        ctx_p = uhnsw.Context(0)
        ctx_p.load_graphs(wl.base, gp, g2, variant=uhnsw.VARIANT_PGRAPH, graph_p=pv)
        first = {}
        for name, c in (("U-HNSW", ctx), ("HNSW on G_p", ctx_p)):
            for ef in efs:
                r = run(p_all, 10, ef, ctx=c)
                row = dict(p=pv, method=name, ef=ef, recall_at_10=r["recall"], qps=r["qps"], walk_ms=r["walk_ms"],
                           verify_ms=r["verify_ms"], mean_n_p=r["mean_n_p"], mean_n_b=r["mean_n_b"])
                out["per_p_hnsw"]["rows"].append(row)
                log("per-p", json.dumps(row))
                if r["recall"] >= TARGET_RECALL:
                    first[name] = row
                    break
        ctx_p.close()
        u, h = first.get("U-HNSW"), first.get("HNSW on G_p")
        out["per_p_hnsw"]["summary"].append(dict(
            p=pv, u_hnsw_ef=u and u["ef"], u_hnsw_qps=u and u["qps"], hnsw_ef=h and h["ef"],
            hnsw_qps=h and h["qps"], u_hnsw_over_hnsw=round(u["qps"] / h["qps"], 3) if u and h else None,
            graph_build_s=round(gp.seconds, 1)))
        log("per-p summary", json.dumps(out["per_p_hnsw"]["summary"][-1]))
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ef", type=int, default=0, help="skip calibration, use this efSearch")
    ap.add_argument("--forms", default="fp32,bf16-batched,fp32-batched",
                    help="comma list of fp32, bf16-batched, fp32-batched, fp16-batched")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-host-api", action="store_true",
                    help="skip the host-pointer (PCIe-inclusive) leg of the FP32 form")
    ap.add_argument("--workload", type=int, default=2, choices=(2, 3, 4, 5, 7),
                    help="2: the headline workload; 3: precision form; 4: batching form; "
                         "5: serving form (10,000,000 x 96, graphs built on the GPU); 7: the headline vectors on "
                         "the extended index (G_0.5 + G_1, p over 0.2..1.0)")
    ap.add_argument("--sweep", action="store_true",
                    help="method diagnostics on the headline workload instead of the benchmark: the "
                         "verification ablation, the t / tau study and per-graph recall across p")
    ap.add_argument("--reduced", action="store_true",
                    help="--workload 5 at 1,000,000 of its 10,000,000 rows (CPU-built graphs)")
    ap.add_argument("--knobs", default="",
                    help="with --ef: the batched forms' launch knobs instead of the autotuner's, as "
                         "beam_width=2,visited_slots=2048,waves_per_block=1,persistent=3,waves_per_cu=0")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device (a kernel of known traffic for counter scaling)")
    a = ap.parse_args()
    knobs = {}
    for kv in filter(None, a.knobs.split(",")):
        key, val = kv.split("=")
        if key not in ("beam_width", "visited_slots", "waves_per_block", "persistent", "waves_per_cu"):
            ap.error(f"--knobs: unknown knob {key}")
        knobs[key] = int(val)
    if knobs and not a.ef:
        ap.error("--knobs needs --ef")
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the query path runs on a single MI355X and the library has no "
              "multi-GPU path (replicate the index per GPU and shard queries to scale).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import synth.graphs as sg
    from paper_2605_02030_amd import uhnsw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.sweep:
        run_sweep(a, torch, uhnsw, sg, synth)
        return
    if a.workload not in (2, 7):
        run_secondary(a, torch, uhnsw, sg, synth)
        return
    ext = a.workload == 7
    variant = uhnsw.VARIANT_EXT if ext else uhnsw.VARIANT_STD
    t0 = time.time()
    wl = synth.make_workload(a.workload)
    log(f"workload {wl.name}: n={wl.n} d={wl.d} nq={wl.nq} ({time.time() - t0:.1f}s)")
    gt = dict(np.load(GT_PATH)) if not ext else gt_for(wl)
    if bytes(gt["digest"]).decode() != wl.digest():
        raise SystemExit("ground-truth file does not match the generated workload")
    t0 = time.time()
    g1, g2 = sg.build_graphs(wl, cache=True, verbose=True, extended=ext)
    log(f"graphs ready in {time.time() - t0:.1f}s")

    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x 1 GiB device copies done")
        del src, dst

    forms = {}
    specs = {"fp32": (uhnsw.STORE_F32, 0, 4), "bf16-batched": (uhnsw.STORE_BF16, 1, 2),
             "fp32-batched": (uhnsw.STORE_F32, 1, 4), "fp16-batched": (uhnsw.STORE_F16, 1, 2)}
    runs = {}  # form -> (ef, beam, storage, elem, fused, timing dict)
    probes = None
    for name in [f.strip() for f in a.forms.split(",") if f.strip()]:
        storage, persistent, elem = specs[name]
        f = Form(torch, uhnsw, wl, g1, g2, storage, persistent, name, variant)
        num_cus, rate_khz = f.ctx.device_info()
        if name == "fp32":  # ceiling probes on the resident FP32 rows (512 B per row)
            probes = dict(gather_512B_gbs=round(f.ctx.probe_gather(512), 1),
                          gather_256B_gbs=round(f.ctx.probe_gather(256), 1),
                          exp_log_lane_ops_per_s=float(f"{f.ctx.probe_transcendental():.4g}"),
                          exp_log_peak_lane_ops_per_s=TRANS_PEAK)
            log("probes", json.dumps(probes))
        if a.ef:
            f.set_ef(a.ef, knobs=knobs)
            ef, table = a.ef, []
        else:
            ef, table = calibrate(f, gt, name, EF_GRID_EXT if ext else EF_GRID)
        r = timed(f, a.steps, a.warmup, wl, rate_khz)
        rec = recall_at_k(f.ids.cpu().numpy(), gt["ids"], gt["qidx"])
        qps = wl.nq * a.steps / r["total_s"]
        beam = f.tuned[ef].beam_width if persistent else 1
        forms[name] = dict(ef=ef, beam=beam, recall_at_10=round(rec, 4), qps=round(qps, 1),
                           ms_per_step=round(r["total_s"] * 1e3 / a.steps, 4), p50_ms=round(r["p50_ms"], 4),
                           p99_ms=round(r["p99_ms"], 4), prepass_ms=round(r["prepass_ms"], 4),
                           walk_ms=round(r["walk_ms"], 4), verify_ms=round(r["verify_ms"], 4),
                           walk_reps=r["walk_reps"], walk_ms_median=round(r["walk_ms_median"], 4),
                           walk_ms_range=[round(x, 4) for x in r["walk_ms_range"]],
                           mean_n_b=round(r["n_b"], 1), mean_n_exp=round(r["n_exp"], 1),
                           mean_n_p=round(r["n_p"], 2), flagged=r["flags"], sweep=table)
        if persistent:
            t = f.tuned[ef]
            forms[name].update(streams=f.pipeline, slots=t.visited_slots, wpb=t.waves_per_block,
                               schedule=t.persistent, waves_per_cu=t.waves_per_cu)
        runs[name] = (ef, beam, storage, elem, bool(persistent), r)
        # the host-pointer entry point (PCIe copies in and out included); left
        # out of --copy-probe runs, whose 1 GiB copies must be the only large
        # copy dispatches the counter scaling reads, and of --no-host-api runs
        if name == "fp32" and not a.copy_probe and not a.no_host_api:
            forms[name]["host_api_qps"] = host_api_qps(f, wl, ef, uhnsw)
        log(name, json.dumps(forms[name]))
        f.ctx.close()
        del f
        torch.cuda.empty_cache()

    main_name = "fp32" if "fp32" in forms else next(iter(forms))
    m = forms[main_name]
    serving_out = None
    if not a.no_serving:
        serving_out = serving(torch, uhnsw, wl, g1, g2, gt, m["ef"], variant=variant)
    baseline, counts = None, {}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) and the method's own row counts ...")
        baseline, counts = cpu_baseline(wl, g1, g2, m["ef"], variant=variant,
                                        combos=[(v[0], v[1], v[2]) for v in runs.values()])
        log("cpu baseline", json.dumps(baseline))
    # per form: the method's bytes over the walk kernel's own time; the GPU's
    # rows over the method's rows (re-reads after the visited cache forgot a node)
    for name, (ef, beam, storage, elem, fused, r) in runs.items():
        c = counts.get((ef, beam, storage))
        if c is None:
            continue
        wb, pb = method_bytes(wl, elem, r["stats"], c, fused)
        fm = forms[name]
        fm["method_bytes_per_launch"] = round(wb + pb)
        fm["walk_gbs"] = round(wb / (r["walk_ms"] * 1e-3) / 1e9, 1)
        fm["walk_frac_of_hbm_peak"] = round(wb / (r["walk_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        fm["gpu_rows_over_method_rows"] = round(float(r["stats"]["n_b"].astype(np.float64).sum()
                                                      / c["n_b"].astype(np.float64).sum()), 4)
        if fm.get("streams", 1) > 1:  # per step with two launches in flight
            fm["step_gbs"] = round((wb + pb) / (r["total_s"] / a.steps) / 1e9, 1)
            fm["step_frac_of_hbm_peak"] = round(fm["step_gbs"] / HBM_PEAK_GBS, 4)

    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    kernel_hash = h.hexdigest()[:16]
    with open(HOST_SRC, "rb") as fh:
        host_hash = hashlib.sha256(fh.read()).hexdigest()[:16]
    m = forms[main_name]
    wb_main, _ = (method_bytes(wl, runs[main_name][3], runs[main_name][5]["stats"],
                               counts[runs[main_name][:3]], runs[main_name][4])
                  if runs[main_name][:3] in counts else (None, None))
    walk_s = runs[main_name][5]["walk_ms"] * 1e-3
    if wb_main is None:  # no oracle run: the kernel's own counters (re-reads included)
        st = runs[main_name][5]["stats"]
        wb_main = float((st["n_b"] - st["n_up"]).astype(np.float64).sum() * wl.d * runs[main_name][3]
                        + st["n_exp"].astype(np.float64).sum() * 128)
        bytes_from = "kernel counters (rows re-read after the visited cache forgot them included)"
    else:
        bytes_from = "oracle walk with an exact visited set (method's own rows)"
    ach = wb_main / walk_s / 1e9
    traffic_ok = (kernel_hash == TRAFFIC["kernel_sha256_prefix"] and host_hash == TRAFFIC["host_sha256_prefix"]
                  and m["ef"] == TRAFFIC["ef"] and main_name == "fp32" and not ext)
    out = {
        "metric": "QPS at recall@10>=0.9 under mixed-p L_p (1 GPU)",
        "value": m["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "d": wl.d, "queries_per_step": wl.nq,
                   "k": 10, "p": "grid 0.2..1.0 cycling" if ext else "grid 0.5..2.0 cycling", "M": 16,
                   "efConstruction": 200, "efSearch": m["ef"], "form": main_name,
                   "index": "extended: G_0.5 (L0.5) + G_1, cutoff 0.6" if ext else "G1 (L1) + G2 (L2), cutoff 1.4"},
        "recall_at_10": m["recall_at_10"],
        "p50_ms": m["p50_ms"],
        "p99_ms": m["p99_ms"],
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": TRAFFIC["bytes_per_launch"] if traffic_ok else None,
                     "kernel": "walk_kernel" if main_name == "fp32" else "search_kernel",
                     "kernel_ms": round(walk_s * 1e3, 4), "algorithmic_bytes_per_launch": round(wb_main),
                     "bytes_from": bytes_from,
                     "traffic_over_algorithmic": round(TRAFFIC["bytes_per_launch"] / wb_main, 4)
                     if traffic_ok else None},
        "probes": probes,
        "forms": forms,
    }
    if serving_out is not None:
        out["serving"] = serving_out
    if baseline is not None:
        out["cpu_baseline"] = baseline
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
