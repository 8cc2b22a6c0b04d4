"""Pins of the several-bases oracle (Section 3.A, Algorithm 1; readings R9,
R10) against facts that do not come from the oracle's own formulas:
special bases whose result is exact, reductions to the single-basis search,
the probe-all limit, and a brute-force re-derivation of the candidate set."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_03453_amd import workloads as W


def test_rotation_by_identity_and_permutation_is_exact():
    X = W.tie_heavy(500, 12, seed=71)
    I = np.eye(12, dtype=np.float32)
    XI = O.rotate(X, I)
    # identity: same values (a zero may change sign: 0 + (-0) = +0)
    assert np.array_equal(np.abs(XI), np.abs(X)) and np.array_equal(XI == 0, X == 0)
    assert np.array_equal(XI[X != 0], X[X != 0])
    P = np.eye(12, dtype=np.float32)[np.random.default_rng(3).permutation(12)]
    XP = O.rotate(X, P)
    want = X @ P.T.astype(np.float64)  # each output is one exact product
    assert np.array_equal(np.abs(XP), np.abs(want).astype(np.float32))


def test_rotation_within_fp32_bound_and_norm_preserved():
    X = W.gaussian_db(300, 24, seed=72)
    M = W.random_bases(2, 24, seed=73)[1]
    got = O.rotate(X, M).astype(np.float64)
    exact = X.astype(np.float64) @ M.astype(np.float64).T
    bound = 24 * 2.0 ** -24 * (np.abs(X.astype(np.float64)) @ np.abs(M.astype(np.float64)).T)
    assert (np.abs(got - exact) <= bound).all()
    assert np.allclose(np.linalg.norm(got, axis=1), np.linalg.norm(X, axis=1), rtol=1e-5)
    # the bases are orthonormal
    Q = W.random_bases(4, 24, seed=73).astype(np.float64)
    for q in Q:
        assert np.allclose(q @ q.T, np.eye(24), atol=1e-6)


def test_identity_hash_equals_single_basis_hash():
    X = W.tie_heavy(2000, 10, seed=74)
    ix = O.build_index_rot(X, 2, np.eye(10, dtype=np.float32)[None])
    o = O.build_index(X, 2)
    for k in ("cone", "offsets", "perm"):
        assert np.array_equal(ix["tables"][0][k], o[k])


@pytest.mark.parametrize("B", [1, 40, 700, 5000])
def test_one_identity_basis_is_the_single_basis_search(B):
    X = W.gaussian_db(4000, 12, seed=75)
    Y = W.gaussian_queries(120, 12, seed=76)
    o = O.build_index(X, 2)
    ix = O.build_index_rot(X, 2, np.eye(12, dtype=np.float32)[None])
    a = O.search(X, o, Y, B)
    b = O.search_rot(X, ix, Y, B)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("R,B", [(2, 300), (3, 1000), (4, 77)])
def test_repeated_basis_equals_single_basis_at_divided_budget(R, B):
    # R copies of one basis: each cone is met R times in a row, rows are
    # analyzed once, and the visited count grows R times faster (R10)
    X = W.gaussian_db(3000, 16, seed=77)
    Y = W.gaussian_queries(100, 16, seed=78)
    M = W.random_bases(2, 16, seed=79)[1]
    single = O.build_index_rot(X, 2, M[None])
    rep = O.build_index_rot(X, 2, np.repeat(M[None], R, axis=0))
    a = O.search_rot(X, single, Y, math.ceil(B / R))
    b = O.search_rot(X, rep, Y, B)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_probe_all_is_exhaustive():
    X = W.gaussian_db(1500, 8, seed=80)
    Y = W.gaussian_queries(60, 8, seed=81)
    ix = O.build_index_rot(X, 2, W.random_bases(3, 8, seed=82))
    idx, d32, d64, nca = O.search_rot(X, ix, Y, 10 ** 9)
    i32, e32, i64, e64 = O.exhaustive(X, Y)
    assert np.array_equal(idx, i32) and np.array_equal(d32, e32)
    assert (nca == 1500).all()


def test_brute_force_candidate_set():
    # re-derive, with sets, the rows Algorithm 1 analyzes within the budget
    X = W.gaussian_db(800, 6, seed=83)
    Y = W.gaussian_queries(40, 6, seed=84)
    rots = W.random_bases(3, 6, seed=85)
    ix = O.build_index_rot(X, 2, rots)
    for B in (30, 150):
        idx, d32, d64, nca = O.search_rot(X, ix, Y, B)
        for q in range(len(Y)):
            seen, visited, done = set(), 0, False
            walks = [O.walk(O.rotate(Y[q:q + 1], rots[r])[0], 2) for r in range(3)]
            for lvl in range(len(walks[0])):
                for r in range(3):
                    t = ix["tables"][r]
                    c = walks[r][lvl]
                    rows = t["perm"][t["offsets"][c]:t["offsets"][c + 1]]
                    seen.update(int(v) for v in rows)
                    visited += len(rows)
                    if visited >= B:
                        done = True
                        break
                if done:
                    break
            assert nca[q] == len(seen)
            cand = np.array(sorted(seen))
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in seen
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)
