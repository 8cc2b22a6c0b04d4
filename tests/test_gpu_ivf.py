"""GPU parity of the coarse-cluster path (ROSANNA+, Section 4.B; reading R12)
through the C ABI.  k-means: the centroids after every iteration count are
bit-identical to the oracle's (the assignments are exact FP32 decisions and
both sides sum a cluster's rows in float64 in ascending row order).  Clustered
tables and searches: with the oracle's centroids on both sides, bucket ids,
residual tops, offsets, permutation, result rows, FP32 distances and
candidate counts are bit-exact."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import dev, say, unpack_top

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


@pytest.mark.parametrize("kind", ["gauss", "desc", "patch"])
def test_kmeans_bit_exact(orc, kind):
    if kind == "gauss":
        X = W.gaussian_db(8000, 16, seed=6101) * 2
    elif kind == "desc":
        X = W.sift_like_db(6000, 128, seed=6102)
    else:
        X = W.patch_rows(W.patch_field(128))
    C = 24
    init = np.ascontiguousarray(X[:: len(X) // C][:C]).astype(np.float32)
    for iters in (0, 1, 5):
        say(f"[ivf] k-means {kind} N={len(X)} D={X.shape[1]} C={C} iters={iters}")
        g = B.os_ann_kmeans(dev(X), dev(init), iters)
        torch.cuda.synchronize()
        o = orc.kmeans(X, init, iters)
        assert np.array_equal(g.cpu().numpy().view(np.uint32), o.view(np.uint32)), (kind, iters)


def check_ivf(orc, X, Y, L, cent, nprobes, budgets, tag):
    say(f"[ivf] table {tag} N={X.shape[0]} D={X.shape[1]} C={len(cent)} L={L} Q={Y.shape[0]}")
    h = B.os_ann_build_ivf(dev(X), L, dev(cent), nprobes[0])
    o = orc.build_index_ivf(X, L, cent)
    try:
        ex = B.os_ann_export(h)
        torch.cuda.synchronize()
        cone = ex["cone"].cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(cone, o["cone"]), tag
        ti, ts = unpack_top(ex["top"].cpu().numpy().view(np.uint64), L)
        assert np.array_equal(ti, o["top"]) and np.array_equal(ts, o["sign"]), tag
        assert np.array_equal(ex["offsets"].cpu().numpy(), o["offsets"]), tag
        assert np.array_equal(ex["perm"].cpu().numpy(), o["perm"]), tag
        yq = dev(Y)
        for npb in nprobes:
            B.os_ann_set_nprobe(h, npb)
            for budget in budgets:
                gi, gd, gn = B.os_ann_search_ex(h, yq, budget)
                torch.cuda.synchronize()
                oi, od32, od64, on = orc.search_ivf(X, o, Y, budget, npb)
                assert np.array_equal(gn.cpu().numpy(), on), (tag, npb, budget)
                assert np.array_equal(gi.cpu().numpy(), oi), (tag, npb, budget)
                assert np.array_equal(gd.cpu().numpy().view(np.uint32), od32.view(np.uint32)), (tag, npb, budget)
    finally:
        B.os_ann_free(h)


def test_ivf_gaussian(orc):
    X = W.gaussian_db(10000, 16, seed=6103) * 2
    Y = W.gaussian_queries(300, 16, seed=6104) * 2
    cent = orc.kmeans(X, X[:32], 4)
    check_ivf(orc, X, Y, 2, cent, (1, 3, 8), (1, 50, 600, 10 ** 9), "gauss d16 C32")


def test_ivf_sift_like_and_patches(orc):
    X = W.sift_like_db(20000, 128, seed=6105)
    Y, _ = W.descriptor_queries(X, 200)
    cent = orc.kmeans(X, X[::1000][:16], 3)
    check_ivf(orc, X, Y, 2, cent, (1, 4), (100, 2000), "sift-like u8 C16")
    img = W.patch_field(128)
    Xp = W.patch_rows(img)
    Yimg = np.roll(img, (3, 5), axis=(0, 1)) + np.random.default_rng(13).normal(0, 0.05, img.shape)
    Yp = W.patch_rows(Yimg)[::61]
    cent = orc.kmeans(Xp, np.ascontiguousarray(Xp[::2000][:8]).astype(np.float32), 3)
    check_ivf(orc, Xp, Yp, 2, cent, (2,), (40, 900), "patches f16 C8")


def test_ivf_one_cluster_at_the_origin_is_the_plain_table(orc):
    X = W.gaussian_db(5000, 12, seed=6106)
    Y = W.gaussian_queries(150, 12, seed=6107)
    h1 = B.os_ann_build_ex(dev(X), 2)
    hc = B.os_ann_build_ivf(dev(X), 2, dev(np.zeros((1, 12), dtype=np.float32)), 1)
    try:
        for budget in (1, 100, 2000):
            a = B.os_ann_search_ex(h1, dev(Y), budget)
            b = B.os_ann_search_ex(hc, dev(Y), budget)
            torch.cuda.synchronize()
            for u, v in zip(a, b):
                assert torch.equal(u, v)
    finally:
        B.os_ann_free(h1)
        B.os_ann_free(hc)


def test_ivf_empty_clusters(orc):
    # a far centroid holds no row: queries near it search an empty cluster
    X = W.gaussian_db(3000, 8, seed=6108)
    cent = np.concatenate([orc.kmeans(X, X[:4], 2), np.full((1, 8), 100.0, dtype=np.float32)])
    Y = np.concatenate([W.gaussian_queries(40, 8, seed=6109), np.full((3, 8), 99.0, dtype=np.float32)])
    check_ivf(orc, X, Y, 2, cent, (1, 2), (20, 400), "empty cluster")


def test_ivf_errors():
    X = W.gaussian_db(500, 8, seed=6110)
    cent = dev(X[:4].copy())
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_ivf(dev(X), 2, cent, 5)  # nprobe > C
    assert e.value.code == B.OS_ANN_EINVAL
    h = B.os_ann_build_ivf(dev(X), 2, cent, 2)
    try:
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_set_nprobe(h, 0)
        assert e.value.code == B.OS_ANN_EINVAL
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_search_ex(h, dev(W.gaussian_queries(3, 8, seed=1)), 10, mode=B.OS_ANN_MODE_TILED)
        assert e.value.code == B.OS_ANN_ENOTSUP
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_classify(h, dev(W.gaussian_queries(3, 8, seed=1)), 10)
        assert e.value.code == B.OS_ANN_ENOTSUP
        i, d, n = B.os_ann_search_ex(h, dev(np.zeros((0, 8), dtype=np.float32)), 10)
        assert i.numel() == 0
    finally:
        B.os_ann_free(h)
