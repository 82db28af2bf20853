"""Pins for the oracle's L_p distance and brute-force ground truth.

The L_p distance of the problem statement (U-HNSW paper, Sec. 1.1 and
Sec. 2.1) is the Minkowski form. Pins: textbook closed forms for the
paper's cheap classes p = 1, 2 (add/sub/mul) and p = 0.5, 1.5 (square
root), library routines (torch.cdist, scipy minkowski), and the norm
inequalities behind the paper's norm-equivalence argument (Sec. 3.1).
"""
import numpy as np
import pytest
import scipy.spatial.distance as ssd
import torch

import oracle


@pytest.fixture(scope="module")
def pairs():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((40, 37)).astype(np.float32)
    q = rng.standard_normal((40, 37)).astype(np.float32)
    return x, q


def test_closed_forms(pairs):
    x, q = pairs
    for xi, qi in zip(x, q):
        dlt = np.abs(xi.astype(np.float64) - qi.astype(np.float64))
        assert oracle.lp_dist(xi, qi, 1.0) == pytest.approx(np.linalg.norm(dlt, 1), rel=1e-13)
        assert oracle.lp_dist(xi, qi, 2.0) == pytest.approx(np.linalg.norm(dlt, 2), rel=1e-13)
        assert oracle.lp_dist(xi, qi, 0.5) == pytest.approx(np.sum(np.sqrt(dlt)) ** 2, rel=1e-13)
        assert oracle.lp_dist(xi, qi, 1.5) == pytest.approx(
            np.sum(dlt * np.sqrt(dlt)) ** (2.0 / 3.0), rel=1e-13)
        # un-rooted sums
        assert oracle.lp_sum(xi, qi, 0.5) == pytest.approx(np.sum(np.sqrt(dlt)), rel=1e-13)
        assert oracle.lp_sum(xi, qi, 2.0) == pytest.approx(np.sum(dlt * dlt), rel=1e-13)


def test_integer_data_exact():
    rng = np.random.Generator(np.random.PCG64(4))
    x = rng.integers(0, 256, size=128).astype(np.float32)
    q = rng.integers(0, 256, size=128).astype(np.float32)
    dlt = np.abs(x.astype(np.int64) - q.astype(np.int64))
    assert oracle.lp_sum(x, q, 1.0) == float(dlt.sum())
    assert oracle.lp_sum(x, q, 2.0) == float((dlt * dlt).sum())


def test_library_cdist(pairs):
    x, q = pairs
    # 0.2 and 0.3: the extended variant's range (Sec. 4.5)
    for p in (0.2, 0.3, 0.5, 0.73, 1.0, 1.37, 1.5, 2.0):
        ref_t = torch.cdist(torch.from_numpy(x).double(), torch.from_numpy(q).double(), p=p).numpy()
        for i in range(0, 40, 7):
            for j in range(0, 40, 9):
                got = oracle.lp_dist(x[i], q[j], p)
                assert got == pytest.approx(ref_t[i, j], rel=1e-12)
                assert got == pytest.approx(ssd.minkowski(x[i].astype(np.float64),
                                                          q[j].astype(np.float64), p), rel=1e-12)


def test_identity_and_symmetry(pairs):
    x, q = pairs
    for p in (0.5, 0.8, 1.3, 2.0):
        assert oracle.lp_dist(x[0], x[0], p) == 0.0
        assert oracle.lp_dist(x[1], q[1], p) == oracle.lp_dist(q[1], x[1], p)


def test_metric_inequalities():
    rng = np.random.Generator(np.random.PCG64(5))
    pts = rng.standard_normal((30, 11)).astype(np.float32)
    for p in (0.5, 0.6, 0.9, 1.0, 1.4, 2.0):
        for a in range(0, 30, 3):
            for b in range(1, 30, 4):
                for c in range(2, 30, 5):
                    dab, dbc, dac = (oracle.lp_dist(pts[u], pts[w], p) for u, w in ((a, b), (b, c), (a, c)))
                    if p >= 1:
                        assert dac <= (dab + dbc) * (1 + 1e-12)  # triangle inequality
                    else:
                        # S_p is subadditive for p < 1, and the quasi-metric bound
                        sab, sbc, sac = (oracle.lp_sum(pts[u], pts[w], p) for u, w in ((a, b), (b, c), (a, c)))
                        assert sac <= (sab + sbc) * (1 + 1e-12)
                        assert dac <= 2 ** (1 / p - 1) * (dab + dbc) * (1 + 1e-12)


def test_norm_ordering():
    """||v||_q <= ||v||_p <= d^(1/p - 1/q) ||v||_q for p <= q."""
    rng = np.random.Generator(np.random.PCG64(6))
    z = np.zeros(23, np.float32)
    for _ in range(20):
        v = rng.standard_normal(23).astype(np.float32)
        for p, q in ((0.5, 1.0), (0.7, 1.3), (1.0, 2.0), (1.5, 2.0), (0.5, 2.0)):
            np_, nq_ = oracle.lp_dist(v, z, p), oracle.lp_dist(v, z, q)
            assert nq_ <= np_ * (1 + 1e-12)
            assert np_ <= 23 ** (1 / p - 1 / q) * nq_ * (1 + 1e-12)


def test_bruteforce_vs_cdist():
    rng = np.random.Generator(np.random.PCG64(8))
    base = rng.standard_normal((700, 19)).astype(np.float32)
    qs = rng.standard_normal((9, 19)).astype(np.float32)
    ps = np.array([0.5, 0.6, 0.77, 1.0, 1.2, 1.4, 1.5, 1.8, 2.0], np.float32)
    ids, S = oracle.bruteforce(base, qs, ps, 10)
    for i in range(9):
        dd = torch.cdist(torch.from_numpy(qs[i:i + 1]).double(), torch.from_numpy(base).double(),
                         p=float(ps[i])).numpy()[0]
        order = np.lexsort((np.arange(700), dd))[:10]
        assert list(ids[i]) == list(order)
        np.testing.assert_allclose(S[i] ** (1 / float(ps[i])), dd[order], rtol=1e-12)


def test_bruteforce_ties_by_id():
    """Integer data has exact ties; the smaller id must come first."""
    base = np.array([[3], [1], [5], [1], [3], [7]], np.float32)
    q = np.array([[2]], np.float32)
    for p in (0.5, 1.0, 2.0):
        ids, S = oracle.bruteforce(base, q, np.float32(p), 4)
        assert list(ids[0]) == [0, 1, 3, 4]  # all at |delta| = 1; ids ascending
    ids, S = oracle.bruteforce(base, q, np.float32(1.0), 8)  # K > n pads
    assert list(ids[0][6:]) == [-1, -1] and np.isinf(S[0][6:]).all()
