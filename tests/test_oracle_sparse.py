"""Pins of the sparse table (Section 4: a second-level hash table when the
cones are very many; reading R15) against facts that do not come from its
own lookups: where the dense table fits it is exactly the dense table with
the empty cones left out and both search the same; at N_C far beyond any
dense table (K = 64, G = 5: 2.4e8 cones) the keys are the distinct hashed
cones found by numpy, and the candidate sets are re-derived by brute force
from the walk's first positions and a dictionary of cone sizes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_03453_amd import workloads as W


@pytest.mark.parametrize("K,G", [(12, 2), (16, 3), (8, 4)])
def test_equals_the_dense_table_without_empty_cones(K, G):
    X = W.gaussian_db(5000, K, seed=191 + K)
    Y = W.gaussian_queries(70, K, seed=192 + K)
    d = O.build_index(X, G)
    s = O.build_index_sparse(X, G)
    sizes = np.diff(d["offsets"])
    ne = np.flatnonzero(sizes)
    assert np.array_equal(s["keys"], ne)
    assert np.array_equal(s["offsets"], np.append(d["offsets"][ne], len(X)))
    assert np.array_equal(s["perm"], d["perm"])
    for B in (1, 37, 900, 5000, 10 ** 6):
        for u, v in zip(O.search_sparse(X, s, Y, B), O.search(X, d, Y, B)):
            assert np.array_equal(u, v)
    for C in (1, 4, 60, d["n_cones"] + 1):
        for u, v in zip(O.search_sparse(X, s, Y, C, cones=True), O.search(X, d, Y, C, cones=True)):
            assert np.array_equal(u, v)


def _big():
    X = W.gaussian_db(20000, 64, seed=193)
    Y = W.gaussian_queries(25, 64, seed=194)
    return X, Y, O.build_index_sparse(X, 5)


def test_large_table_keys_and_rows():
    X, Y, s = _big()
    assert s["n_cones"] == 7624512 * 32
    cone = O.hash_rows(X, 5)[2]
    keys, counts = np.unique(cone, return_counts=True)
    assert np.array_equal(s["keys"], keys)
    assert np.array_equal(np.diff(s["offsets"]), counts)
    order = np.lexsort((np.arange(len(X)), cone))
    assert np.array_equal(s["perm"], order)


def test_large_table_brute_force_candidates():
    X, Y, s = _big()
    cone = O.hash_rows(X, 5)[2]
    rows_of = {}
    for n, c in enumerate(cone):
        rows_of.setdefault(int(c), []).append(n)
    for B, cones in ((1, True), (40, True), (1, False), (3, False)):
        idx, d32, d64, nca = O.search_sparse(X, s, Y, B, cones=cones)
        for q in range(len(Y)):
            cand = []
            if cones:
                for c in O.walk_prefix(Y[q], 5, B):
                    cand += rows_of.get(int(c), [])
            else:
                n = 1 << 12
                while True:  # a long enough walk prefix to meet the budget
                    pre = O.walk_prefix(Y[q], 5, n)
                    total, take = 0, []
                    for c in pre:
                        r = rows_of.get(int(c), [])
                        take += r
                        total += len(r)
                        if r and total >= B:
                            break
                    if total >= B or len(pre) < n:
                        break
                    n *= 4
                cand = take
            assert nca[q] == len(cand)
            if not cand:
                assert idx[q] == -1 and np.isinf(d32[q])
                continue
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in cand
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


def test_large_table_every_row():
    X, Y, s = _big()
    idx, d32, d64, nca = O.search_sparse(X, s, Y[:5], len(X))
    i32, e32, i64, e64 = O.exhaustive(X, Y[:5])
    assert np.array_equal(idx, i32) and np.array_equal(d32, e32)
    assert (nca == len(X)).all()


def test_walk_cap():
    # a budget the first 2^22 walk positions cannot meet stops there (R15)
    X, Y, s = _big()
    cap = 1 << 22
    keys, off = s["keys"], s["offsets"]
    for B, cones in ((5000, False), (cap * 2, True)):
        idx, d32, d64, nca = O.search_sparse(X, s, Y[:2], B, cones=cones)
        for q in range(2):
            pre = O.walk_prefix(Y[q], 5, cap)
            assert len(pre) == cap
            at = np.searchsorted(keys, pre)
            hit = (at < len(keys)) & (keys[np.minimum(at, len(keys) - 1)] == pre)
            rows = np.concatenate([s["perm"][off[u]:off[u + 1]] for u in at[hit]])
            assert nca[q] == len(rows) and len(rows) < 5000
            dd = ((X[rows].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in set(rows.tolist())
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)
