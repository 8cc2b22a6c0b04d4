"""Pins of the coarse-cluster oracle (ROSANNA+, Section 4.B; reading R12)
against facts that do not come from its own formulas: k-means on
well-separated blobs recovers the blob means, the assignment agrees with a
float64 brute force away from ties, one cluster centred at the origin is the
plain search, probing every cluster with an unbounded budget is exhaustive
search, and a brute-force re-derivation of the candidate set."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_03453_amd import workloads as W


def _blobs(n_per=400, C=6, K=8, seed=121):
    r = np.random.default_rng(seed)
    centres = r.normal(0.0, 20.0, (C, K))
    X = np.concatenate([centres[c] + r.normal(0.0, 1.0, (n_per, K)) for c in range(C)])
    perm = r.permutation(len(X))
    return X[perm].astype(np.float32), centres


def test_kmeans_recovers_blob_means():
    X, centres = _blobs()
    # one seed point inside every blob (the first row of each), 10 iterations
    truth = O.assign(X, centres.astype(np.float32))
    init = np.stack([X[np.flatnonzero(truth == c)[0]] for c in range(len(centres))])
    cent = O.kmeans(X, init, 10)
    for c in range(len(centres)):
        members = X[truth == c].astype(np.float64)
        assert np.allclose(cent[c], members.mean(0), atol=1e-4)


def test_kmeans_zero_iterations_and_empty_cluster():
    X, centres = _blobs(n_per=50, C=3)
    init = np.concatenate([X[:3], np.full((1, X.shape[1]), 1e6, dtype=np.float32)])
    assert np.array_equal(O.kmeans(X, init, 0), init)
    cent = O.kmeans(X, init, 2)
    assert np.array_equal(cent[3], init[3])  # nothing is ever assigned to the far centroid


def test_assignment_matches_float64_brute_force():
    X = W.gaussian_db(2000, 10, seed=122)
    cent = W.gaussian_queries(16, 10, seed=123)
    a = O.assign(X, cent)
    d = ((X.astype(np.float64)[:, None, :] - cent.astype(np.float64)[None]) ** 2).sum(2)
    srt = np.sort(d, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-4 * srt[:, 1]
    assert np.array_equal(a[clear], d.argmin(1)[clear])


@pytest.mark.parametrize("B", [1, 60, 900])
def test_one_cluster_at_the_origin_is_the_plain_search(B):
    X = W.gaussian_db(3000, 12, seed=124)
    Y = W.gaussian_queries(80, 12, seed=125)
    ix = O.build_index_ivf(X, 2, np.zeros((1, 12), dtype=np.float32))
    o = O.build_index(X, 2)
    for k in ("offsets", "perm"):
        assert np.array_equal(ix[k], o[k])
    for u, v in zip(O.search(X, o, Y, B), O.search_ivf(X, ix, Y, B, 1)):
        assert np.array_equal(u, v)


def test_every_cluster_unbounded_is_exhaustive():
    X = W.gaussian_db(1200, 8, seed=126)
    Y = W.gaussian_queries(40, 8, seed=127)
    cent = O.kmeans(X, X[:5], 3)
    ix = O.build_index_ivf(X, 2, cent)
    idx, d32, d64, nca = O.search_ivf(X, ix, Y, 10 ** 9, 5)
    i32, e32, i64, e64 = O.exhaustive(X, Y)
    assert np.array_equal(idx, i32) and np.array_equal(d32, e32)
    assert (nca == 1200).all()


def test_cluster_search_brute_force():
    X = W.gaussian_db(1500, 8, seed=128) * 3
    Y = W.gaussian_queries(40, 8, seed=129) * 3
    cent = O.kmeans(X, X[::300][:5], 4)
    ix = O.build_index_ivf(X, 2, cent)
    nc = ix["n_cones"]
    for B, nprobe in ((30, 2), (200, 3)):
        idx, d32, d64, nca = O.search_ivf(X, ix, Y, B, nprobe)
        Bc = math.ceil(B / nprobe)
        for q in range(len(Y)):
            dc = ((cent.astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            near = np.argsort(dc, kind="stable")[:nprobe]
            cand = []
            for c in near:
                r = (Y[q] - cent[c]).astype(np.float32)
                total = 0
                for cone in O.walk(r, 2):
                    b = c * nc + cone
                    rows = ix["perm"][ix["offsets"][b]:ix["offsets"][b + 1]]
                    if len(rows) == 0:
                        continue
                    cand.extend(int(v) for v in rows)
                    total += len(rows)
                    if total >= Bc:
                        break
            assert nca[q] == len(cand)
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in cand
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)
