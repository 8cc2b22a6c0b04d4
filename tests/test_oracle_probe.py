"""Pins of the oracle's probe order and budget rule (Section 3.B, Alg. 1).

Pinned: every cone is visited exactly once; the first cone is the query's
own; phase A visits every profile once with the query's signs in
non-decreasing paper profile distance; at G=1 phase A is the argsort of |y|;
the candidate count is the smallest whole-cone prefix reaching the budget.
Parity unpinned (a reading, the paper prints no probe list): the order among
profiles at equal distance, and the order of the sign-flipped cones."""
import numpy as np
import pytest

from paper_1509_03453_amd import workloads as W
from tests.paper_defs import colex_subsets, decode_cone, profile_distance, sign_bits


@pytest.mark.parametrize("K,G", [(3, 1), (3, 2), (6, 2), (8, 3), (16, 1), (16, 2), (7, 7)])
def test_walk_visits_every_cone_once(orc, K, G):
    Y = W.gaussian_queries(5, K, seed=40 + K + G)
    Y[0, 0] = -0.0
    nc = orc.num_cones(K, G)
    table = colex_subsets(K, G)
    n_prof = len(table)
    for y in Y:
        order = np.argsort(-np.abs(y), kind="stable")
        w = orc.walk(y, G)
        assert sorted(w.tolist()) == list(range(nc))
        _, _, own = orc.hash_rows(y[None, :], G)
        assert w[0] == own[0]
        ys = sign_bits(y)
        dists, flips = [], []
        for k, c in enumerate(w):
            prof, signs = decode_cone(c, K, G, table)
            nflip = sum(int(s != ys[i]) for s, i in zip(signs, prof))
            flips.append(nflip)
            if k < n_prof:
                assert nflip == 0
                dists.append(profile_distance(prof, order, G))
        # phase A: every profile once, distance non-decreasing
        assert len({decode_cone(c, K, G, table)[0] for c in w[:n_prof]}) == n_prof
        assert all(a <= b for a, b in zip(dists, dists[1:]))
        # phase B: number of flipped signs non-decreasing
        assert all(a <= b for a, b in zip(flips, flips[1:]))
        if G == 1:
            assert [decode_cone(c, K, 1, table)[0][0] for c in w[:K]] == order.tolist()


@pytest.mark.parametrize("B", [1, 7, 100, 512, 2000, 10 ** 9])
def test_budget_is_smallest_whole_cone_prefix(orc, B):
    X = W.gaussian_db(4000, 8, seed=51)
    idx = orc.build_index(X, 2)
    off = idx["offsets"]
    sizes = np.diff(off)
    for y in W.gaussian_queries(20, 8, seed=52):
        probes, ncand = orc.probe(y, 2, off, B)
        w = orc.walk(y, 2)
        cum = np.cumsum(sizes[w])
        hit = np.flatnonzero(cum >= B)
        stop = hit[0] if hit.size else len(w) - 1
        want = [c for c in w[:stop + 1] if sizes[c] > 0]
        assert probes.tolist() == want
        assert ncand == (cum[stop] if hit.size else 4000)
        assert ncand >= min(B, 4000)
