"""GPU parity of the fixed-C mode (Section 3, Table III; reading R13: each
walk takes its first C cones, empty ones included) through the C ABI flag
OS_ANN_FLAG_BUDGET_CONES, against the oracle's fixed-C searches on the same
seeded inputs.

FP32 mode (one basis, several bases, keyed PCA table, clustered table):
result rows, FP32 distances and candidate counts are bit-exact.  Tiled mode:
candidate counts are bit-exact, the reported distance is the exact FP32
distance of the reported row, and a differing row must be explained by a
near tie at the R-th screening value.  Walks whose cones are all empty
report row -1, distance +inf and no candidate."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import candidates_of, check_screened, dev, say

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


def run(h, yq, C, mode=B.OS_ANN_MODE_FP32, R=8):
    gi, gd, gn = B.os_ann_search_ex(h, yq, C, mode=mode, rerank_r=R, cones=True)
    torch.cuda.synchronize()
    return gi.cpu().numpy(), gd.cpu().numpy(), gn.cpu().numpy()


def same_fp32(g, o, tag):
    gi, gd, gn = g
    oi, od32, od64, on = o
    assert np.array_equal(gn, on), tag
    assert np.array_equal(gi, oi), tag
    assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), tag


def same_tiled(orc, X, Y, g, o, tag, max_mismatch=0.02, index=None, C=None):
    cand = candidates_of(orc, index, Y, C, cones=True) if index is not None else None
    check_screened(orc, X, Y, g, o, tag, max_mismatch=max_mismatch, is_candidate=cand)


@pytest.mark.parametrize("kind", ["gauss", "desc", "patch"])
def test_cones_one_basis(orc, kind):
    if kind == "gauss":
        X = W.gaussian_db(20000, 16, seed=7101)
        Y = W.gaussian_queries(515, 16, seed=7102)
        L = 2
    elif kind == "desc":
        X = W.descriptor_db(12000, 128)
        Y, _ = W.descriptor_queries(X, 333)
        L = 2
    else:
        X, Y = W.patch_pair(96)
        Y = Y[::7][:450]
        L = 2
    say(f"[cones] one basis {kind} N={len(X)} D={X.shape[1]} Q={len(Y)} dtype={X.dtype}")
    h = B.os_ann_build_ex(dev(X), L)
    o = orc.build_index(X, L)
    nc = o["n_cones"]
    yq = dev(Y)
    try:
        for C in (1, 3, 64, 700, nc, nc + 9):
            say(f"[cones] {kind} fp32 C={C}")
            same_fp32(run(h, yq, C), orc.search(X, o, Y, C, cones=True), (kind, C))
        for C in (1, 5, 64, 500):
            say(f"[cones] {kind} tiled C={C}")
            same_tiled(orc, X, Y, run(h, yq, C, B.OS_ANN_MODE_TILED),
                       orc.search_tiled(X, o, Y, C, R=8, cones=True), (kind, "tiled", C), index=o, C=C)
    finally:
        B.os_ann_free(h)


def test_cones_empty_walks(orc):
    # 300 rows over 180 cones: C = 1 leaves some walks without a candidate
    X = W.gaussian_db(300, 10, seed=7103)
    Y = W.gaussian_queries(130, 10, seed=7104)
    say("[cones] empty walks N=300 D=10")
    h = B.os_ann_build_ex(dev(X), 2)
    o = orc.build_index(X, 2)
    yq = dev(Y)
    try:
        for C in (1, 2):
            g = run(h, yq, C)
            assert (g[2] == 0).any()
            same_fp32(g, orc.search(X, o, Y, C, cones=True), ("empty", C))
            same_tiled(orc, X, Y, run(h, yq, C, B.OS_ANN_MODE_TILED),
                       orc.search_tiled(X, o, Y, C, R=8, cones=True), ("empty tiled", C), index=o, C=C)
    finally:
        B.os_ann_free(h)


def test_cones_several_bases(orc):
    X = W.gaussian_db(12000, 16, seed=7105)
    Y = W.gaussian_queries(301, 16, seed=7106)
    rots = W.random_bases(3, 16, seed=7107)
    say("[cones] several bases R=3")
    h = B.os_ann_build_rot(dev(X), 2, dev(np.ascontiguousarray(rots, dtype=np.float32)))
    o = orc.build_index_rot(X, 2, rots)
    yq = dev(Y)
    try:
        for C in (1, 4, 50, 480, 10 ** 6):
            say(f"[cones] several bases C={C}")
            same_fp32(run(h, yq, C), orc.search_rot(X, o, Y, C, cones=True), ("rot", C))
    finally:
        B.os_ann_free(h)


def test_cones_keyed_pca(orc):
    X = W.sift_like_db(10000, 64, seed=7108)
    Y = W.gaussian_queries(257, 64, seed=7109) * 40 + X[:257]
    mu, P, var = orc.pca_basis(X, 12)
    say("[cones] keyed table k=12")
    h = B.os_ann_build_proj(dev(X), 2, dev(P), dev(mu))
    o = orc.build_index_proj(X, 2, mu, P)
    yq = dev(np.ascontiguousarray(Y, dtype=np.float32))
    try:
        for C in (1, 6, 90, 10 ** 5):
            say(f"[cones] keyed C={C}")
            same_fp32(run(h, yq, C), orc.search_proj(X, o, Y.astype(np.float32), C, cones=True), ("pca", C))
    finally:
        B.os_ann_free(h)


def test_cones_clusters(orc):
    X = W.gaussian_db(9000, 16, seed=7110) * 3
    Y = W.gaussian_queries(263, 16, seed=7111) * 3
    cent = orc.kmeans(X, X[::900][:10], 3)
    say("[cones] clusters C=10")
    h = B.os_ann_build_ivf(dev(X), 2, dev(cent), 1)
    o = orc.build_index_ivf(X, 2, cent)
    yq = dev(Y)
    try:
        for npb in (1, 3):
            B.os_ann_set_nprobe(h, npb)
            for C in (1, 7, 120, 10 ** 4):
                say(f"[cones] clusters nprobe={npb} C={C}")
                same_fp32(run(h, yq, C), orc.search_ivf(X, o, Y, C, npb, cones=True), ("ivf", npb, C))
    finally:
        B.os_ann_free(h)


def test_cones_graph_and_workspace(orc):
    # the same call as a cone count and as a row budget, replayed from
    # graphs with the same pointers: each replays its own launch sequence
    X = W.gaussian_db(8000, 16, seed=7112)
    Y = W.gaussian_queries(200, 16, seed=7113)
    h = B.os_ann_build_ex(dev(X), 2)
    o = orc.build_index(X, 2)
    yq = dev(Y)
    s = torch.cuda.Stream()
    nb = max(B.os_ann_workspace_bytes(h, 200, 40, cones=c) for c in (True, False))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    oi = torch.empty(200, dtype=torch.int64, device="cuda")
    od = torch.empty(200, dtype=torch.float32, device="cuda")
    on = torch.empty(200, dtype=torch.int64, device="cuda")
    refs = {c: orc.search(X, o, Y, 40, cones=c) for c in (True, False)}
    try:
        for rep in range(3):
            for cones in (True, False):
                say(f"[cones] graph replay {rep} cones={cones}")
                oi.fill_(-7)
                od.fill_(-1.0)
                on.fill_(-1)
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    B.os_ann_search_ex(h, yq, 40, stream=s, workspace=ws, out_idx=oi, out_dist=od, out_ncand=on,
                                       flags=B.OS_ANN_FLAG_GRAPH, cones=cones)
                s.synchronize()
                junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
                torch.cuda.synchronize()
                del junk
                g = (oi.cpu().numpy(), od.cpu().numpy(), on.cpu().numpy())
                same_fp32(g, refs[cones], ("graph", rep, cones))
    finally:
        torch.cuda.synchronize()
        B.os_ann_free(h)
