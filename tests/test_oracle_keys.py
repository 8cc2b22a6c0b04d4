"""Pins of the oracle's hashing (Section 2, eq. (2), Fig. 2)."""
import itertools
import os

import numpy as np
import pytest

from paper_1509_03453_amd import workloads as W
from tests.paper_defs import colex_subsets, decode_cone, sign_bits, top_set_bruteforce

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig2_toy_dataset.txt")


def _fig2():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        vec, p1, c1, p2, c2 = [s.strip() for s in line.split("|")]
        rows.append(([float(t) for t in vec.split()], p1, int(c1), p2, int(c2)))
    return rows


@pytest.mark.parametrize("G,pcol,ccol", [(1, 1, 2), (2, 3, 4)])
def test_fig2_memberships(orc, G, pcol, ccol):
    """Every vector of the toy dataset lands in the profile and cone the
    figure prints for it (left table G=1, right table G=2)."""
    rows = _fig2()
    X = np.array([r[0] for r in rows], dtype=np.float32)
    top, sg, cone = orc.hash_rows(X, G)
    for n, r in enumerate(rows):
        want_prof = tuple(int(t) - 1 for t in r[pcol].split("-"))
        prof, signs = decode_cone(cone[n], 3, G)
        assert prof == want_prof, (n, prof, want_prof)
        c = int("".join(str(s) for s in signs), 2)
        assert c == r[ccol], (n, c, r[ccol])
        assert tuple(sorted(top[n])) == want_prof


def test_fig2_bucket_sizes(orc):
    X = np.array([r[0] for r in _fig2()], dtype=np.float32)
    # G=1: profiles {1},{2},{3} x cones c=0,1
    _, _, c1 = orc.hash_rows(X, 1)
    off1, _ = orc.bucket(c1, orc.num_cones(3, 1))
    assert np.diff(off1).tolist() == [2, 4, 2, 3, 4, 1]
    # G=2: profiles {1,2},{1,3},{2,3} x cones c=0..3
    _, _, c2 = orc.hash_rows(X, 2)
    off2, _ = orc.bucket(c2, orc.num_cones(3, 2))
    assert np.diff(off2).tolist() == [2, 1, 1, 5, 1, 0, 2, 0, 0, 1, 1, 2]


def test_num_cones_closed_forms(orc):
    """N_C = C(K,G) 2^G: 6 and 12 for the toy set, "almost 30000" for K=16,
    G=4, 2K for G=1, 2K(K-1) for G=2, 2^K for G=K (Section 2)."""
    assert orc.num_cones(3, 1) == 6 and orc.num_cones(3, 2) == 12
    assert orc.num_cones(16, 4) == 29120
    for K in (2, 5, 16, 64, 128):
        assert orc.num_cones(K, 1) == 2 * K
        assert orc.num_cones(K, 2) == 2 * K * (K - 1)
    for K in (1, 3, 8, 16):
        assert orc.num_cones(K, K) == 2 ** K


@pytest.mark.parametrize("K,G", [(3, 1), (3, 2), (5, 2), (6, 3), (7, 4), (8, 8), (9, 1)])
def test_cone_encoding_bijective(orc, K, G):
    """For every profile and sign pattern, a vector whose G largest |v_i| sit
    on that profile with those signs hashes to colex(profile)*2^G + bits,
    and the map is onto [0, N_C)."""
    table = colex_subsets(K, G)
    vecs, want = [], []
    for rank, S in enumerate(table):
        for bits in range(1 << G):
            v = np.full(K, 0.5, dtype=np.float32)
            for j, i in enumerate(S):
                mag = 10.0 + (j * 7 % G)  # distinct large magnitudes
                neg = not ((bits >> (G - 1 - j)) & 1)
                v[i] = -mag if neg else mag
            vecs.append(v)
            want.append(rank * (1 << G) + bits)
    _, _, cone = orc.hash_rows(np.array(vecs), G)
    assert cone.tolist() == want
    assert sorted(cone.tolist()) == list(range(orc.num_cones(K, G)))


def test_top1_is_first_argmax(orc):
    """G=1 reduces to the first index of max |x| (BLAS i?amax semantics)."""
    X = W.tie_heavy(4000, 13, seed=11)
    top, sg, cone = orc.hash_rows(X, 1)
    assert np.array_equal(top[:, 0], np.argmax(np.abs(X), axis=1))
    assert np.array_equal(sg[:, 0], sign_bits(X[np.arange(len(X)), top[:, 0]]))
    assert np.array_equal(cone, 2 * top[:, 0] + sg[:, 0])


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("G", [1, 2, 3, 5])
def test_topG_is_stable_argsort(orc, G, dtype):
    """General G: the first G entries of a stable argsort of -|x|."""
    X = W.tie_heavy(3000, 11, seed=12 + G).astype(dtype)
    top, sg, cone = orc.hash_rows(X, G)
    want = np.argsort(-np.abs(X.astype(np.float32)), axis=1, kind="stable")[:, :G]
    assert np.array_equal(top, want)
    assert np.array_equal(sg, sign_bits(np.take_along_axis(X, want, 1)))


def test_uint8_rows(orc):
    """uint8 rows hash like their float values; every sign bit is 1."""
    X = W.descriptor_db(2000, 32, seed=5)
    t8, s8, c8 = orc.hash_rows(X, 2)
    tf, sf, cf = orc.hash_rows(X.astype(np.float32), 2)
    assert np.array_equal(t8, tf) and np.array_equal(c8, cf)
    assert (s8 == 1).all()


def test_negative_zero_is_nonnegative(orc):
    """Fig. 2 caption: c=0 holds x<0, c=1 the others, so -0.0 and 0.0 give 1."""
    X = np.array([[0.0, 0.0], [-0.0, 0.0], [-0.0, -0.0], [0.0, -1.0]], dtype=np.float32)
    top, sg, cone = orc.hash_rows(X, 1)
    assert top[:, 0].tolist() == [0, 0, 0, 1]
    assert sg[:, 0].tolist() == [1, 1, 1, 0]


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_tiny_with_ties(orc, seed):
    """Brute force over every G-subset on tiny tie-heavy inputs, all G."""
    r = np.random.default_rng(seed)
    K = int(r.integers(1, 7))
    X = W.tie_heavy(48, K, seed=100 + seed)
    for G in range(1, K + 1):
        top, sg, cone = orc.hash_rows(X, G)
        table = colex_subsets(K, G)
        for n in range(X.shape[0]):
            S = top_set_bruteforce(X[n], G)
            prof, signs = decode_cone(cone[n], K, G, table)
            assert prof == S
            assert signs == tuple(int(b) for b in sign_bits(X[n, list(S)]))
            assert set(top[n].tolist()) == set(S)
