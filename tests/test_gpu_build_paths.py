"""The build's and the tiled search's size-dependent paths, each against the oracle.

* The stable radix sort of the rows by cone: one block of 1024 threads holds
  up to 16,384 keys in LDS; above that the multi-block passes run.  Both
  sides of the boundary must give the oracle's permutation (rows of one
  cone in ascending original order), bucket offsets and permuted rows.
* A build that also makes the low-precision copy takes the table's closing
  check at the copy's end and sizes the copy by the bound N + 15 min(cones,
  N) when that bound is within a quarter of N, else by the exact count read
  back first; the copy's layout is one block's work for up to 65,536 cones
  and several launches above.  Tiled searches on such builds must pass the
  screened comparison with the oracle (Section 3, reading R7).
"""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import candidates_of, check_screened, dev, gpu_index, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


@pytest.mark.parametrize("N", [16383, 16384, 16385])
def test_sort_boundary(orc, N):
    # 480 cones (D = 16, L = 2): about 34 rows per cone, so every bucket
    # holds ties that the sort must keep in ascending row order
    X = W.gaussian_db(N, 16, seed=5100 + N % 7)
    say(f"[build] sort boundary N={N}")
    h, g = gpu_index(X, 2)
    try:
        o = orc.build_index(X, 2)
        assert np.array_equal(g["cone"], o["cone"]), N
        assert np.array_equal(g["offsets"], o["offsets"]), N
        assert np.array_equal(g["perm"], o["perm"]), N
        rows = B.os_ann_export_rows(h).cpu().numpy()
        assert np.array_equal(rows, X[o["perm"]]), N
    finally:
        B.os_ann_free(h)


@pytest.mark.parametrize("case", ["bound", "exact", "many_cones"])
def test_lowp_build_paths(orc, case):
    R = 8
    if case == "bound":  # 32 cones, 200,000 rows: the copy sized by the bound
        X, Y, L, budget = W.gaussian_db(200000, 16, seed=5201), W.gaussian_queries(300, 16, seed=5202), 1, 20000
    elif case == "exact":  # 1984 cones, 30,000 rows: the exact count read first
        X, Y, L, budget = W.gaussian_db(30000, 32, seed=5203), W.gaussian_queries(300, 32, seed=5204), 2, 3000
    else:  # 333,312 cones (D = 64, L = 3): the copy's layout in several launches
        X, Y, L, budget = W.gaussian_db(20000, 64, seed=5205), W.gaussian_queries(150, 64, seed=5206), 3, 1000
    say(f"[build] lowp {case} N={X.shape[0]} D={X.shape[1]} L={L} budget={budget}")
    h = B.os_ann_build_ex(dev(X), L, want_lowp=True)
    try:
        info = B.os_ann_info(h)
        o = orc.build_index(X, L)
        assert info["n_nonempty"] == int((np.diff(o["offsets"]) > 0).sum()), case
        gi, gd, gn = B.os_ann_search_ex(h, dev(Y), budget, mode=B.OS_ANN_MODE_TILED, rerank_r=R)
        torch.cuda.synchronize()
        gi, gd, gn = gi.cpu().numpy(), gd.cpu().numpy(), gn.cpu().numpy()
        oi, od32, od64, on, dtr, top = orc.search_tiled(X, o, Y, budget, R=R)
        check_screened(orc, X, Y, (gi, gd, gn), (oi, od32, od64, on, dtr, top), (case, budget),
                       is_candidate=candidates_of(orc, o, Y, budget))
    finally:
        B.os_ann_free(h)
