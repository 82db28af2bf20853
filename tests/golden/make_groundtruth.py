"""Write the exact L_p ground truth used for recall@10 on the 1M x 128
mixture workload: tests/golden/gt_mixture-1M-d128.npz.

Calls only the oracle's brute force (FP64, ties by smaller id; the recall
definition of the U-HNSW paper, Sec. 4.1.2) on the seeded inputs from
``synth``. The sample is every 5th query (2,000 of 10,000): 5 is coprime to
the 16-value p grid, so each p in {0.5, ..., 2.0} appears 125 times.

    python tests/golden/make_groundtruth.py [--threads N]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gt_mixture-1M-d128.npz")
STRIDE = 5
K = 10


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    wl = synth.make_workload(2)
    qidx = np.arange(0, wl.nq, STRIDE, dtype=np.int32)
    t0 = time.time()
    ids = np.empty((len(qidx), K), np.int32)
    S = np.empty((len(qidx), K), np.float64)
    step = 100
    for s in range(0, len(qidx), step):
        sel = qidx[s:s + step]
        ids[s:s + step], S[s:s + step] = oracle.bruteforce(wl.base, wl.queries[sel], wl.p[sel], K, a.threads)
        print(f"{s + len(sel)}/{len(qidx)} queries, {time.time() - t0:.0f}s", flush=True)
    np.savez(OUT, qidx=qidx, ids=ids, S=S, p=wl.p[qidx], K=np.int32(K),
             digest=np.frombuffer(wl.digest().encode(), np.uint8))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
