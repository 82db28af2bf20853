"""Write the exact L_p ground truth used for recall@10:
tests/golden/gt_<workload>.npz.

Calls only the oracle's brute force (FP64, ties by smaller id; the recall
definition of the U-HNSW paper, Sec. 4.1.2) on the seeded inputs from
``synth``. Samples:
  workload 2 (mixture-1M-d128): every 5th query (2,000 of 10,000); 5 is
      coprime to the 16-value p grid, so each p appears 125 times;
  workload 3 (gammafeat-1M-d960): every 10th query (100 of 1,000);
  workload 4 (unitgauss-1.18M-d100): every 30th query starting at 1 (the
      K = 10 queries; 334 of 10,000);
  workload 5 at n = 1,000,000 (unitgauss-1M-d96, the serving form's shape
      at a tenth of its size), and with --full at its n = 10,000,000
      (unitgauss-10M-d96): every 10th query (200 of 2,000);
  workload 7 (mixture-1M-d128-pext, the extended variant's p over 0.2..1.0):
      every 10th query (1,000 of 10,000; 10 is coprime to the 9-value grid).

    python tests/golden/make_groundtruth.py [--workload 2|3|4|5|7] [--threads N]

With ``--ideal`` it prints (no file) the idealized recall behind the
graph-choice cutoff (Sec. 3.2, Fig. 2): for the sweep's 200 queries, the
share of the exact L_p top-K found among the exact top-t under the base
metric L1 or L2, for each p of SWEEP_P and t in IDEAL_T (needs the sweep
file).

With ``--sweep`` it writes tests/golden/gt_sweep_<workload>.npz instead: the
top-50 of every 50th query of workload 2 (200 queries) under each p of
SWEEP_P, the paper's 0.1 grid over [0.5, 2] plus its ablation value 0.51
(Sec. 4.4), each query taking every p (the diagnostics of the parameter
and ablation sweeps).
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE = {2: (0, 5), 3: (0, 10), 4: (1, 30), 5: (0, 10), 7: (0, 10)}  # workload -> (first query, stride)
SIZE = {5: 1_000_000}  # workload -> reduced n
K = 10
SWEEP_P = np.array([0.5, 0.51] + [round(0.6 + 0.1 * i, 1) for i in range(15)], np.float32)
SWEEP_K = 50
IDEAL_T = (10, 30, 60, 100, 200, 300)


def ideal(a):
    wl = synth.make_workload(2)
    gt = dict(np.load(os.path.join(HERE, f"gt_sweep_{wl.name}.npz")))
    if bytes(gt["digest"]).decode() != wl.digest():
        raise SystemExit("sweep ground truth does not match the generated workload")
    qidx = gt["qidx"]
    T = max(IDEAL_T)
    base_top = {}
    for metric in (1.0, 2.0):  # exact top-T under the base metric (L_1, L_2)
        ids = np.empty((len(qidx), T), np.int32)
        for s in range(0, len(qidx), 50):
            sel = qidx[s:s + 50]
            ids[s:s + 50], _ = oracle.bruteforce(wl.base, wl.queries[sel], np.full(len(sel), metric, np.float32), T,
                                                 a.threads)
        base_top[metric] = ids
    out = {"workload": wl.name, "queries": len(qidx), "t": list(IDEAL_T), "rows": []}
    for j, pv in enumerate(gt["p"]):
        for K in (10, 50):
            row = {"p": round(float(pv), 2), "K": K}
            for metric, name in ((1.0, "L1"), (2.0, "L2")):
                rec = []
                for t in IDEAL_T:
                    hit = [len(set(gt["ids"][j, i, :K].tolist()) & set(base_top[metric][i, :t].tolist())) / K
                           for i in range(len(qidx))]
                    rec.append(round(float(np.mean(hit)), 4))
                row[name] = rec
            out["rows"].append(row)
    import json

    print(json.dumps(out))


def sweep(a):
    wl = synth.make_workload(2)
    qidx = np.arange(0, wl.nq, 50, dtype=np.int32)
    out = os.path.join(HERE, f"gt_sweep_{wl.name}.npz")
    t0 = time.time()
    ids = np.empty((len(SWEEP_P), len(qidx), SWEEP_K), np.int32)
    S = np.empty((len(SWEEP_P), len(qidx), SWEEP_K), np.float64)
    for j, pv in enumerate(SWEEP_P):
        for s in range(0, len(qidx), 50):
            sel = qidx[s:s + 50]
            p = np.full(len(sel), pv, np.float32)
            ids[j, s:s + 50], S[j, s:s + 50] = oracle.bruteforce(wl.base, wl.queries[sel], p, SWEEP_K, a.threads)
        print(f"p={pv:.2f} done, {time.time() - t0:.0f}s", flush=True)
    np.savez(out, qidx=qidx, p=SWEEP_P, ids=ids, S=S, K=np.int32(SWEEP_K),
             digest=np.frombuffer(wl.digest().encode(), np.uint8))
    print("wrote", out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--workload", type=int, default=2, choices=sorted(SAMPLE))
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--ideal", action="store_true")
    ap.add_argument("--full", action="store_true",
                    help="workload 5 at its full n = 10,000,000 (gt_unitgauss-10M-d96.npz)")
    a = ap.parse_args()
    if a.sweep:
        return sweep(a)
    if a.ideal:
        return ideal(a)
    wl = synth.make_workload(a.workload, n=None if a.full else SIZE.get(a.workload))
    first, stride = SAMPLE[a.workload]
    qidx = np.arange(first, wl.nq, stride, dtype=np.int32)
    out = os.path.join(HERE, f"gt_{wl.name}.npz")
    t0 = time.time()
    ids = np.empty((len(qidx), K), np.int32)
    S = np.empty((len(qidx), K), np.float64)
    step = 50
    for s in range(0, len(qidx), step):
        sel = qidx[s:s + step]
        ids[s:s + step], S[s:s + step] = oracle.bruteforce(wl.base, wl.queries[sel], wl.p[sel], K, a.threads)
        print(f"{s + len(sel)}/{len(qidx)} queries, {time.time() - t0:.0f}s", flush=True)
    np.savez(out, qidx=qidx, ids=ids, S=S, p=wl.p[qidx], K=np.int32(K),
             digest=np.frombuffer(wl.digest().encode(), np.uint8))
    print("wrote", out)


if __name__ == "__main__":
    main()
