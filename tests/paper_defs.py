"""Independent restatements of the paper's definitions, used only to pin the
oracle (none of this is imported by the oracle or the GPU library).

Everything here is built from Python's itertools / numpy library routines so
that a mistake in the oracle's own encoding cannot cancel out."""
from __future__ import annotations

import itertools

import numpy as np


def colex_subsets(K: int, G: int):
    """All G-subsets of range(K) listed in colexicographic order."""
    return sorted(itertools.combinations(range(K), G), key=lambda s: s[::-1])


def decode_cone(cone: int, K: int, G: int, table=None):
    """cone id -> (profile as a sorted tuple, sign bits per profile member)."""
    table = table if table is not None else colex_subsets(K, G)
    rank, bits = divmod(int(cone), 1 << G)
    prof = table[rank]
    signs = tuple((bits >> (G - 1 - j)) & 1 for j in range(G))
    return prof, signs


def sign_bits(v) -> np.ndarray:
    """1 unless the value is negative (zero and -0.0 count as non-negative)."""
    return (~(np.asarray(v) < 0)).astype(np.int64)


def top_set_bruteforce(v, G: int):
    """The unique G-subset S whose members all precede every non-member in
    decreasing |v| with ties to the lower index (found by enumeration)."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    K = a.shape[0]
    found = []
    for S in itertools.combinations(range(K), G):
        ok = all((a[i] > a[j]) or (a[i] == a[j] and i < j)
                 for i in S for j in range(K) if j not in S)
        if ok:
            found.append(S)
    assert len(found) == 1
    return found[0]


def profile_distance(prof, query_order, G: int) -> int:
    """Paper Section 3.B: G minus the level of the closest common ancestor of
    the profile and the query's profile on the query's chain of ancestors
    {i1}, {i1,i2}, ... (members of a profile ranked by the query's order)."""
    rank = {int(c): r for r, c in enumerate(query_order)}
    members = sorted(prof, key=lambda c: rank[c])
    level = 0
    for g in range(1, G + 1):
        if set(members[:g]) == set(int(c) for c in query_order[:g]):
            level = g
        else:
            break
    return G - level


def fp32_seq_dist(x, y) -> np.float32:
    """Squared distance in float32, i ascending, each op rounded (numpy scalars)."""
    acc = np.float32(0.0)
    for a, b in zip(np.asarray(x, np.float32), np.asarray(y, np.float32)):
        d = np.float32(a - b)
        acc = np.float32(acc + np.float32(d * d))
    return acc
