"""Helpers of the GPU parity tests: move arrays, call the C ABI through the
binding, decode its packed outputs.  Nothing here computes the method."""
import sys

import numpy as np
import torch

from paper_1509_03453_amd import binding as B


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def unpack_top(packed: np.ndarray, L: int):
    p = packed.astype(np.uint64)
    idx = np.stack([((p >> np.uint64(9 * j)) & np.uint64(0xFF)).astype(np.int64) for j in range(L)], 1)
    sg = np.stack([((p >> np.uint64(9 * j + 8)) & np.uint64(1)).astype(np.uint8) for j in range(L)], 1)
    return idx, sg


def gpu_index(X: np.ndarray, L: int):
    """Build through the C ABI; returns (handle, exported arrays as numpy)."""
    h = B.os_ann_build_ex(dev(X), L)
    ex = B.os_ann_export(h)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in ex.items()}
    out["cone"] = out["cone"].view(np.uint32).astype(np.int64)
    out["top_idx"], out["top_sign"] = unpack_top(out["top"].view(np.uint64), L)
    return h, out


def gpu_search(h, Y: np.ndarray, budget: int, mode=B.OS_ANN_MODE_FP32):
    i, d, n = B.os_ann_search_ex(h, dev(Y), budget, mode=mode)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy(), n.cpu().numpy()


# (tag, differing rows, compared queries) of every screened comparison, printed
# at the end of the session by conftest.py
MISMATCHES = []


def candidates_of(orc, index, Y, budget, cones=False, Yk=None):
    """``is_candidate(q, row)``: row lies in one of the cones query q's walk
    takes within the budget (reading R5; R13 with ``cones``).  ``Yk``: the
    keys a keyed table's walk runs on."""
    walk_rows = Y if Yk is None else Yk
    seen = {}

    def is_candidate(q, row):
        if q not in seen:
            y = np.asarray(walk_rows[q], dtype=np.float32)
            pr = (orc.probe_cones(y, index["G"], index["offsets"], budget) if cones
                  else orc.probe(y, index["G"], index["offsets"], budget))
            seen[q] = set(pr[0].tolist())
        return int(index["cone"][row]) in seen[q]
    return is_candidate


def check_screened(orc, X, Y, g, o, tag, max_mismatch=0.02, is_candidate=None):
    """Compare a tiled-mode result ``g = (idx, dist, ncand)`` with the
    oracle's screened search ``o = (idx, d32, d64, ncand, dtilde_R, top)``.

    Exact: candidate counts; empty searches give -1 / +inf; the distance is
    the exact FP32 distance of the returned row.  The GPU accumulates d~ in
    FP32 on the matrix cores and the oracle in double, so the R survivors
    may differ where a d~ lies within rounding of the R-th one.  A returned
    row that differs from the oracle's is accepted only when both sides of
    the difference are explained that way:
      * if the row is not among the oracle's R survivors, its d~ lies within
        rounding of the oracle's R-th d~ (the GPU kept a boundary row);
      * if the row is worse than the oracle's by (FP32 distance, row), the
        GPU dropped the oracle's pick, so that pick's d~ lies within
        rounding of the R-th d~; if it is better, it can not be among the
        oracle's survivors (the oracle would have returned it).
    With ``is_candidate`` a differing row must also be a candidate of its
    query (in one of the cones its walk takes).  Such queries must be rare;
    their count is recorded and printed."""
    U = 2.0 ** -24
    gi, gd, gn = g
    oi, od32, od64, on, dtr, top = o
    assert np.array_equal(gn, on), tag
    empty = on == 0
    assert (gi[empty] == -1).all() and np.isinf(gd[empty]).all(), tag
    full = np.flatnonzero(~empty)
    assert ((gi[full] >= 0) & (gi[full] < X.shape[0])).all(), tag
    assert np.array_equal(gd[full].view(np.uint32), orc.pair_d32(X, Y[full], gi[full]).view(np.uint32)), tag
    f16 = X.dtype == np.float16
    D = X.shape[1]
    bad = [q for q in full if gi[q] != oi[q]]
    for q in bad:
        if is_candidate is not None:
            assert is_candidate(q, int(gi[q])), (tag, q, "the returned row is not a candidate of the query")
        xs = orc.round_short(X[[gi[q], oi[q], top[q][-1]]].astype(np.float32), f16).reshape(3, D)
        ys = orc.round_short(Y[q].astype(np.float32), f16)
        tol = 4 * (D + 2) * U * ((xs ** 2).sum(1) + 2 * np.abs(xs * ys).sum(1)).max()
        dg = orc.pair_dtilde(X, Y[q:q + 1], [gi[q]], f16)[0]
        do = orc.pair_dtilde(X, Y[q:q + 1], [oi[q]], f16)[0]
        if gi[q] not in top[q]:
            assert dg <= dtr[q] + tol, (tag, q, "GPU kept a row beyond the R-th d~")
        if (float(gd[q]), int(gi[q])) > (float(od32[q]), int(oi[q])):
            assert do >= dtr[q] - tol, (tag, q, "oracle's pick dropped without a near tie")
        else:
            assert gi[q] not in top[q], (tag, q, "a better survivor the oracle did not return")
    MISMATCHES.append((str(tag), len(bad), len(full)))
    say(f"[screened] {tag}: {len(bad)}/{len(full)} rows differ from the oracle (near ties at the R-th d~)")
    assert len(bad) <= max_mismatch * len(full) + 1, (tag, len(bad))
    return len(bad)
