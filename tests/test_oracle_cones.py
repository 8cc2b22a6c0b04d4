"""Pins of the fixed-C mode (Section 3 and Table III: the search visits a
fixed number C of cones per basis; reading R13: empty cones count, the
budget is per basis and per searched cluster) against facts that do not come
from its own stopping rule: C = 1 is the query's own cone as hashed by the
key function, C = N_C is exhaustive search, C cones match the row-budget
search whose budget is the rows those cones hold, the candidate sets grow
with C, one identity basis and one cluster at the origin reduce to the plain
search, and brute-force re-derivations of the candidate sets."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_03453_amd import workloads as W


def _sizes(ix):
    return np.diff(ix["offsets"])


def test_one_cone_is_the_own_cone():
    X = W.gaussian_db(3000, 10, seed=141)
    Y = W.gaussian_queries(100, 10, seed=142)
    ix = O.build_index(X, 2)
    own = O.hash_rows(Y, 2)[2]
    sz = _sizes(ix)
    for q in range(len(Y)):
        probes, nca = O.probe_cones(Y[q], 2, ix["offsets"], 1)
        assert nca == sz[own[q]]
        assert list(probes) == ([own[q]] if sz[own[q]] else [])
    idx, d32, d64, nca = O.search(X, ix, Y, 1, cones=True)
    assert np.array_equal(nca, sz[own])
    for q in np.flatnonzero(nca):
        rows = ix["perm"][ix["offsets"][own[q]]:ix["offsets"][own[q] + 1]]
        dd = ((X[rows].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
        assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


def test_every_cone_is_exhaustive():
    X = W.gaussian_db(1500, 8, seed=143)
    Y = W.gaussian_queries(50, 8, seed=144)
    ix = O.build_index(X, 2)
    for C in (ix["n_cones"], ix["n_cones"] + 7):
        idx, d32, d64, nca = O.search(X, ix, Y, C, cones=True)
        i32, e32, i64, e64 = O.exhaustive(X, Y)
        assert np.array_equal(idx, i32) and np.array_equal(d32, e32)
        assert (nca == len(X)).all()


@pytest.mark.parametrize("C", [2, 5, 17, 60])
def test_cones_match_the_row_budget_they_hold(C):
    # the row-budget walk with B = the rows of the first C cones stops at the
    # last non-empty one of them: the same candidates, the same answer
    X = W.gaussian_db(4000, 12, seed=145)
    Y = W.gaussian_queries(80, 12, seed=146)
    ix = O.build_index(X, 2)
    a = O.search(X, ix, Y, C, cones=True)
    for q in range(len(Y)):
        if a[3][q] == 0:
            continue
        b = O.search(X, ix, Y[q:q + 1], int(a[3][q]))
        for u, v in zip(a, b):
            assert u[q] == v[0]


def test_candidate_sets_grow_with_c():
    X = W.tie_heavy(2000, 8, seed=147)
    Y = W.gaussian_queries(30, 8, seed=148)
    ix = O.build_index(X, 3)
    sz = _sizes(ix)
    for q in range(len(Y)):
        prev = set()
        for C in (1, 2, 3, 8, 40, 200):
            probes, nca = O.probe_cones(Y[q], 3, ix["offsets"], C)
            assert prev <= set(probes)
            assert nca == sz[probes].sum()
            assert all(sz[probes] > 0)
            prev = set(probes)


def test_brute_force_first_cones():
    X = W.gaussian_db(900, 6, seed=149)
    Y = W.gaussian_queries(40, 6, seed=150)
    ix = O.build_index(X, 2)
    sz = _sizes(ix)
    for C in (3, 11, 40):
        idx, d32, d64, nca = O.search(X, ix, Y, C, cones=True)
        for q in range(len(Y)):
            cones = [c for c in O.walk(Y[q], 2)[:C] if sz[c] > 0]
            cand = np.concatenate([ix["perm"][ix["offsets"][c]:ix["offsets"][c + 1]] for c in cones])
            assert nca[q] == len(cand)
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in set(cand.tolist())
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


@pytest.mark.parametrize("C", [1, 6, 50])
def test_one_identity_basis_and_one_origin_cluster_are_the_plain_search(C):
    X = W.gaussian_db(3000, 12, seed=151)
    Y = W.gaussian_queries(80, 12, seed=152)
    o = O.build_index(X, 2)
    rot = O.build_index_rot(X, 2, np.eye(12, dtype=np.float32)[None])
    ivf = O.build_index_ivf(X, 2, np.zeros((1, 12), dtype=np.float32))
    a = O.search(X, o, Y, C, cones=True)
    for b in (O.search_rot(X, rot, Y, C, cones=True), O.search_ivf(X, ivf, Y, C, 1, cones=True)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_several_bases_brute_force_levels():
    X = W.gaussian_db(800, 6, seed=153)
    Y = W.gaussian_queries(30, 6, seed=154)
    rots = W.random_bases(3, 6, seed=155)
    ix = O.build_index_rot(X, 2, rots)
    for C in (1, 4, 20):
        idx, d32, d64, nca = O.search_rot(X, ix, Y, C, cones=True)
        for q in range(len(Y)):
            seen = set()
            for r in range(3):
                t = ix["tables"][r]
                for c in O.walk(O.rotate(Y[q:q + 1], rots[r])[0], 2)[:C]:
                    seen.update(int(v) for v in t["perm"][t["offsets"][c]:t["offsets"][c + 1]])
            assert nca[q] == len(seen)
            if not seen:
                continue
            cand = np.array(sorted(seen))
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in seen
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


def test_clusters_brute_force_first_cones():
    X = W.gaussian_db(1500, 8, seed=156) * 3
    Y = W.gaussian_queries(30, 8, seed=157) * 3
    cent = O.kmeans(X, X[::300][:5], 4)
    ix = O.build_index_ivf(X, 2, cent)
    nc = ix["n_cones"]
    for C, nprobe in ((2, 2), (15, 3)):
        idx, d32, d64, nca = O.search_ivf(X, ix, Y, C, nprobe, cones=True)
        for q in range(len(Y)):
            dc = ((cent.astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            cand = []
            for c in np.argsort(dc, kind="stable")[:nprobe]:
                for cone in O.walk((Y[q] - cent[c]).astype(np.float32), 2)[:C]:
                    b = c * nc + cone
                    cand.extend(int(v) for v in ix["perm"][ix["offsets"][b]:ix["offsets"][b + 1]])
            assert nca[q] == len(cand)
            if not cand:
                assert idx[q] == -1
                continue
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in cand
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


def test_screened_search_takes_the_same_candidates():
    X = W.gaussian_db(3000, 16, seed=158)
    Y = W.gaussian_queries(60, 16, seed=159)
    ix = O.build_index(X, 2)
    for C in (1, 9, 70):
        a = O.search(X, ix, Y, C, cones=True)
        t = O.search_tiled(X, ix, Y, C, R=8, cones=True)
        assert np.array_equal(a[3], t[3])
        # the screened answer is a candidate whose distance is at least the arg-min's
        has = a[3] > 0
        assert (t[2][has] >= a[2][has]).all()


def test_empty_cones_give_no_candidate():
    # 300 rows over 180 cones: some queries' own cones are empty
    X = W.gaussian_db(300, 10, seed=160)
    Y = W.gaussian_queries(80, 10, seed=161)
    ix = O.build_index(X, 2)
    empty = _sizes(ix)[O.hash_rows(Y, 2)[2]] == 0
    assert empty.any()
    for res in (O.search(X, ix, Y, 1, cones=True), O.search_tiled(X, ix, Y, 1, cones=True)):
        assert np.array_equal(res[3] == 0, empty)
        assert (res[0][empty] == -1).all() and np.isinf(res[1][empty]).all()
        assert (res[0][~empty] >= 0).all()
