"""Pins of the PCA front-end of the oracle (Section 4.B; reading R11) against
facts that do not come from the oracle's own formulas: data built with
known principal axes and variances, projections that are exact, the FP32
error bound of the projection, the reduction of the keyed search to the
plain one, and a brute-force re-derivation of the keyed candidate set."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_03453_amd import workloads as W

U = 2.0 ** -24


def _hadamard(n):
    h = np.ones((1, 1))
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    return h


def _constructed(N=4096, K=12, sig=(8.0, 4.0, 2.0, 1.0), seed=91):
    # rows = mu + sum_i sig_i h_i q_i with h_i distinct non-constant Hadamard
    # columns (zero mean, mutually orthogonal over the N rows): the covariance
    # is exactly sum_i sig_i^2 q_i q_i^T, so the axes are the q_i
    Q = W.random_bases(2, K, seed=seed)[1].astype(np.float64)  # rows orthonormal
    H = _hadamard(N)
    mu = np.arange(K, dtype=np.float64) * 0.5 - 2.0
    X = mu[None, :].repeat(N, 0)
    for i, s in enumerate(sig):
        X = X + s * H[:, 1 + 3 * i][:, None] * Q[i][None, :]
    return X.astype(np.float32), Q, np.asarray(sig) ** 2, mu


def test_pca_recovers_constructed_axes_and_variances():
    X, Q, lam_true, mu_true = _constructed()
    mu, P, lam = O.pca_basis(X, 4)
    assert np.allclose(mu, mu_true, atol=1e-5)
    assert np.allclose(lam, lam_true, rtol=1e-5)
    for i in range(4):
        assert abs(float(P[i].astype(np.float64) @ Q[i])) > 1 - 1e-5
        # sign convention: the largest-magnitude component is positive
        j = int(np.argmax(np.abs(P[i])))
        assert P[i, j] > 0


def test_pca_invariants_on_gaussian_data():
    X = W.gaussian_db(3000, 16, seed=92) * np.linspace(3.0, 0.5, 16, dtype=np.float32)[None, :]
    mu, P, lam = O.pca_basis(X, 6)
    P64 = P.astype(np.float64)
    assert np.allclose(P64 @ P64.T, np.eye(6), atol=1e-6)
    assert (np.diff(lam) <= 0).all()
    keys = (X.astype(np.float64) - mu.astype(np.float64)) @ P64.T
    assert np.allclose(keys.mean(0), 0.0, atol=1e-3)
    assert np.allclose(keys.var(0), lam, rtol=1e-4)


def test_projection_exact_cases():
    X = W.tie_heavy(300, 10, seed=93)
    mu = np.arange(10, dtype=np.float32) - 4.0
    keys = O.project(X, mu, np.eye(10, dtype=np.float32))
    assert np.array_equal(keys, X - mu)
    # a signed permutation of k = 6 coordinates: every key is one exact difference
    rng = np.random.default_rng(94)
    rows = rng.permutation(10)[:6]
    P = np.zeros((6, 10), dtype=np.float32)
    P[np.arange(6), rows] = rng.choice([-1.0, 1.0], 6)
    keys = O.project(X, mu, P)
    want = (X - mu)[:, rows] * P[np.arange(6), rows][None, :]
    assert np.array_equal(np.abs(keys), np.abs(want))
    assert np.array_equal(O.project(X, None, np.eye(10, dtype=np.float32)), X)


def test_projection_within_fp32_bound():
    X = W.gaussian_db(400, 24, seed=95)
    mu, P, _ = O.pca_basis(X, 8)
    got = O.project(X, mu, P).astype(np.float64)
    c = X.astype(np.float64) - mu.astype(np.float64)
    exact = c @ P.astype(np.float64).T
    bound = 2 * (24 + 1) * U * (np.abs(c) @ np.abs(P.astype(np.float64)).T) + 1e-30
    assert (np.abs(got - exact) <= bound).all()


@pytest.mark.parametrize("B", [1, 50, 600, 5000])
def test_identity_keys_are_the_plain_search(B):
    X = W.gaussian_db(4000, 12, seed=96)
    Y = W.gaussian_queries(120, 12, seed=97)
    o = O.build_index(X, 2)
    ix = O.build_index_proj(X, 2, None, np.eye(12, dtype=np.float32))
    for k in ("cone", "offsets", "perm"):
        assert np.array_equal(ix[k], o[k])
    for u, v in zip(O.search(X, o, Y, B), O.search_proj(X, ix, Y, B)):
        assert np.array_equal(u, v)


def test_keyed_search_brute_force():
    # re-derive with sets the rows the keyed search analyzes: the query's key
    # gives the cone order, whole non-empty cones are taken until the budget,
    # distances use every component of the original vectors
    X = W.gaussian_db(1500, 10, seed=98) * np.linspace(2.0, 0.5, 10, dtype=np.float32)[None, :]
    Y = W.gaussian_queries(50, 10, seed=99) * np.linspace(2.0, 0.5, 10, dtype=np.float32)[None, :]
    mu, P, _ = O.pca_basis(X, 4)
    ix = O.build_index_proj(X, 2, mu, P)
    Yk = O.project(Y, mu, P)
    for B in (20, 200):
        idx, d32, d64, nca = O.search_proj(X, ix, Y, B)
        for q in range(len(Y)):
            cand, total = [], 0
            for c in O.walk(Yk[q], 2):
                rows = ix["perm"][ix["offsets"][c]:ix["offsets"][c + 1]]
                if len(rows) == 0:
                    continue
                cand.extend(int(v) for v in rows)
                total += len(rows)
                if total >= B:
                    break
            assert nca[q] == len(cand)
            dd = ((X[cand].astype(np.float64) - Y[q].astype(np.float64)) ** 2).sum(1)
            assert idx[q] in cand
            assert d64[q] == pytest.approx(dd.min(), rel=1e-6)


def test_screened_keyed_search_walks_the_keys():
    # identity axes reproduce the plain screened search; with 12 of 32 axes
    # the screened search takes exactly the keyed search's candidates
    X = W.gaussian_db(4000, 16, seed=231)
    Y = W.gaussian_queries(60, 16, seed=232)
    eye = O.build_index_proj(X, 2, None, np.eye(16, dtype=np.float32))
    plain = O.build_index(X, 2)
    for u, v in zip(O.search_tiled(X, eye, Y, 300, R=8), O.search_tiled(X, plain, Y, 300, R=8)):
        assert np.array_equal(u, v)
    X2 = W.sift_like_db(5000, 32, seed=233)
    Y2 = X2[:50].astype(np.float32) + W.gaussian_queries(50, 32, seed=234) * 20
    mu, P, var = O.pca_basis(X2, 12)
    ix = O.build_index_proj(X2, 2, mu, P)
    for B in (50, 700):
        t = O.search_tiled(X2, ix, Y2, B, R=8)
        k = O.search_proj(X2, ix, Y2, B)
        assert np.array_equal(t[3], k[3])
        assert (t[2] >= k[2]).all()  # the screened pick is a candidate, never closer than the arg-min
