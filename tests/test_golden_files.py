"""CPU checks of the stored ground-truth files and of the benchmark's
command line. The ground truth was written by tests/golden/make_groundtruth.py
from the oracle's FP64 brute force; here: each file still matches the inputs
it was computed for (digest of the seeded workload), its rows are ordered by
(S_p, id) as the recall definition needs, and a few rows agree with a numpy
recomputation of S_p."""
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def _rows_ordered(ids, S):
    # ascending S, ties by smaller id
    dS = np.diff(S, axis=-1)
    tie = dS == 0
    return bool((dS >= 0).all() and (np.diff(ids, axis=-1)[tie] > 0).all())


@pytest.mark.parametrize("workload", [2, 7])
def test_ground_truth_matches_inputs(workload):
    wl = synth.make_workload(workload)
    gt = dict(np.load(os.path.join(GOLD, f"gt_{wl.name}.npz")))
    assert bytes(gt["digest"]).decode() == wl.digest()
    assert _rows_ordered(gt["ids"], gt["S"])
    np.testing.assert_array_equal(gt["p"], wl.p[gt["qidx"]])
    for r in (0, len(gt["qidx"]) // 2, len(gt["qidx"]) - 1):  # numpy recomputation of S_p for the stored ids
        i = int(gt["qidx"][r])
        x = wl.base[gt["ids"][r]].astype(np.float64)
        S = (np.abs(x - wl.queries[i].astype(np.float64)) ** float(wl.p[i])).sum(1)
        np.testing.assert_allclose(S, gt["S"][r], rtol=1e-12)


def test_sweep_ground_truth_matches_inputs():
    wl = synth.make_workload(2)
    gt = dict(np.load(os.path.join(GOLD, "gt_sweep_mixture-1M-d128.npz")))
    assert bytes(gt["digest"]).decode() == wl.digest()
    assert gt["ids"].shape == (len(gt["p"]), len(gt["qidx"]), int(gt["K"]))
    assert _rows_ordered(gt["ids"], gt["S"])
    i = int(gt["qidx"][3])
    for j in (0, 1, len(gt["p"]) - 1):
        x = wl.base[gt["ids"][j, 3]].astype(np.float64)
        S = (np.abs(x - wl.queries[i].astype(np.float64)) ** float(gt["p"][j])).sum(1)
        np.testing.assert_allclose(S, gt["S"][j, 3], rtol=1e-12)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
