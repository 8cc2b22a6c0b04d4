"""Pins of the oracle's distances and search (eq. (1), Algorithm 1)."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1509_03453_amd import workloads as W
from tests.paper_defs import fp32_seq_dist

U = 2.0 ** -24  # unit roundoff of FP32


def test_distance_special_cases(orc):
    X = np.eye(6, dtype=np.float32)
    Y = np.eye(6, dtype=np.float32)[[0, 3]]
    # d(e_i, e_j) = 2 for i != j, 0 for i == j
    for q, row in enumerate([0, 3]):
        d64 = orc.pair_d64(X, Y[q:q + 1], [row])
        assert d64[0] == 0.0
        d64 = orc.pair_d64(X, Y[q:q + 1], [(row + 1) % 6])
        assert d64[0] == 2.0
    # integer data: exact integer distances (3-4-5 and 1-2-2-3)
    A = np.array([[3, 0, 4, 0], [1, 2, 2, 0]], dtype=np.float32)
    Z = np.zeros((2, 4), dtype=np.float32)
    assert orc.pair_d64(A, Z, [0, 1]).tolist() == [25.0, 9.0]
    assert orc.pair_d32(A, Z, [0, 1]).tolist() == [25.0, 9.0]
    # symmetry
    R = W.gaussian_db(2, 33, seed=3)
    assert orc.pair_d64(R[:1], R[1:], [0])[0] == orc.pair_d64(R[1:], R[:1], [0])[0]


@pytest.mark.parametrize("K", [1, 5, 16, 64, 128])
def test_distance_within_rounding_bound_of_exact(orc, K):
    """Against exact rational arithmetic: the double value is within
    (K+2) 2^-53 relative and the FP32 value within (K+2) 2^-24 relative
    (recursive summation of non-negative terms), and the FP32 value equals
    an op-by-op float32 evaluation bit for bit."""
    X = W.gaussian_db(12, K, seed=60 + K) * np.float32(3.0)
    Y = W.gaussian_queries(12, K, seed=61 + K)
    rows = np.arange(12)
    d64 = orc.pair_d64(X, Y, rows)
    d32 = orc.pair_d32(X, Y, rows)
    for q in range(12):
        exact = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(X[q], Y[q]))
        ex = float(exact)
        assert abs(d64[q] - ex) <= (K + 2) * 2.0 ** -53 * ex + 1e-300
        assert abs(float(d32[q]) - ex) <= (K + 2) * U * ex
        assert d32[q] == fp32_seq_dist(X[q], Y[q])


def test_probe_all_equals_exhaustive(orc):
    """With a budget of at least N every cone is probed and the result is the
    exact linear-search NN, bit for bit."""
    X = W.gaussian_db(3000, 16, seed=71)
    Y = W.gaussian_queries(200, 16, seed=72)
    for G in (1, 2, 3):
        idx = orc.build_index(X, G)
        i, d32, d64, nca = orc.search(X, idx, Y, B=3000)
        e32, ed32, e64, ed64 = orc.exhaustive(X, Y)
        assert (nca == 3000).all()
        assert np.array_equal(i, e32) and np.array_equal(d32, ed32)
        assert np.allclose(d64, ed64, rtol=1e-5)


def test_search_is_argmin_over_probed_cones(orc):
    """Brute force over the probed candidate set, ties to the lower row id,
    on tie-heavy integer data (many equal distances)."""
    X = W.tie_heavy(600, 6, seed=81)
    Y = W.tie_heavy(60, 6, seed=82)
    idx = orc.build_index(X, 2)
    off, perm = idx["offsets"], idx["perm"]
    for B in (1, 30, 150):
        i, d32, d64, nca = orc.search(X, idx, Y, B=B)
        for q in range(len(Y)):
            probes, ncand = orc.probe(Y[q], 2, off, B)
            cand = np.concatenate([perm[off[c]:off[c + 1]] for c in probes])
            assert len(cand) == ncand == nca[q]
            d = np.array([fp32_seq_dist(X[r], Y[q]) for r in cand])
            best = cand[np.lexsort((cand, d))[0]]
            assert i[q] == best and d32[q] == d.min()
            assert d64[q] == float(((X[best].astype(np.float64) - Y[q]) ** 2).sum())


def test_mixed_storage_types(orc):
    """uint8 and FP16 rows search like their exact float values."""
    X8 = W.descriptor_db(3000, 32, seed=91)
    Y = np.clip(X8[:50].astype(np.float32) + W.gaussian_queries(50, 32, seed=92) * 8, 0, 255)
    idx = orc.build_index(X8, 2)
    a = orc.search(X8, idx, Y, B=200)
    b = orc.search(X8.astype(np.float32), orc.build_index(X8.astype(np.float32), 2), Y, B=200)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    Xh = W.gaussian_db(2000, 16, seed=93).astype(np.float16)
    Yh = W.gaussian_queries(40, 16, seed=94).astype(np.float16)
    a = orc.search(Xh, orc.build_index(Xh, 2), Yh, B=100)
    b = orc.search(Xh.astype(np.float32), orc.build_index(Xh.astype(np.float32), 2),
                   Yh.astype(np.float32), B=100)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_thread_count_does_not_change_results(orc):
    X = W.gaussian_db(5000, 16, seed=95)
    Y = W.gaussian_queries(300, 16, seed=96)
    idx = orc.build_index(X, 1)
    a = orc.search(X, idx, Y, B=300, nthreads=1)
    b = orc.search(X, idx, Y, B=300, nthreads=8)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
