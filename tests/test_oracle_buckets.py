"""Pins of the oracle's bucketing: one cone-bucketed hash table (Section 4)."""
import numpy as np
import pytest
from scipy import stats

from paper_1509_03453_amd import workloads as W


@pytest.mark.parametrize("N,K,G", [(5000, 16, 1), (20000, 64, 2), (3000, 7, 3), (1, 4, 2)])
def test_bucket_library_reduction_and_invariants(orc, N, K, G):
    X = W.gaussian_db(N, K, seed=31 + K)
    idx = orc.build_index(X, G)
    nc = orc.num_cones(K, G)
    off, perm, cone = idx["offsets"], idx["perm"], idx["cone"]
    # library routines: bincount + cumsum, stable argsort
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(np.bincount(cone, minlength=nc))]))
    assert np.array_equal(perm, np.argsort(cone, kind="stable"))
    # invariants: sizes sum to N, perm is a permutation, rows of a bucket
    # carry that bucket's key and ascend in original order
    assert off[-1] == N and off[0] == 0
    assert np.array_equal(np.sort(perm), np.arange(N))
    for c in np.flatnonzero(np.diff(off)):
        rows = perm[off[c]:off[c + 1]]
        assert (cone[rows] == c).all()
        assert (np.diff(rows) > 0).all()


def test_cone_occupancy_uniform_under_symmetry(orc):
    """Section 2: for a perfectly symmetric source every cone is equally
    likely (N_C is then the mean speed-up).  Chi-square on i.i.d. Gaussian
    data, D=16, G=1: 16384 rows over 32 cones, 512 expected per cone."""
    X = W.gaussian_db(16384, 16, seed=W.SEEDS["gauss16_db"])
    idx = orc.build_index(X, 1)
    sizes = np.diff(idx["offsets"])
    chi2, p = stats.chisquare(sizes)
    assert p > 1e-3, (chi2, p)
    assert abs(sizes.mean() - 512) < 1e-9
