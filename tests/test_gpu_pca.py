"""GPU parity of the PCA front-end (Section 4.B; reading R11) through the C
ABI.  Principal axes: the GPU's float64 moments and host Jacobi
diagonalisation against the oracle's float64 numpy decomposition, within
tolerance (different summation orders).  Keyed tables and searches: both
sides take the same (mean, basis) -- the oracle's -- and must agree bit for
bit on cones, packed tops, offsets, permutation, result rows, FP32
distances and candidate counts."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import check_screened, dev, say, unpack_top

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


def _scaled_gauss(n, d, seed):
    return W.gaussian_db(n, d, seed=seed) * np.linspace(3.0, 0.3, d, dtype=np.float32)[None, :]


def check_axes(orc, X, k, tag):
    say(f"[pca] axes {tag} N={X.shape[0]} D={X.shape[1]} k={k} dtype={X.dtype}")
    mu, P, var = B.os_ann_pca(dev(X), k)
    omu, oP, ovar = orc.pca_basis(X, k)
    assert np.allclose(mu, omu, rtol=1e-6, atol=1e-6), tag
    assert np.allclose(var, ovar, rtol=1e-9, atol=1e-12 * ovar[0]), tag
    assert np.allclose(P, oP, atol=1e-5), tag  # same axes, same signs
    assert np.allclose(P.astype(np.float64) @ P.T.astype(np.float64), np.eye(k), atol=1e-5), tag


def test_axes_gaussian_descriptor_patches(orc):
    check_axes(orc, _scaled_gauss(5000, 16, 5101), 6, "gauss d16")
    Xd = W.descriptor_db(20000, 128, seed=5102)
    check_axes(orc, Xd, 16, "desc u8 d128")
    img = W.patch_field(256)
    check_axes(orc, W.patch_rows(img), 16, "patches f16 d64")


def check_proj(orc, X, Y, L, mu, P, budgets, tag):
    say(f"[pca] keyed table {tag} N={X.shape[0]} D={X.shape[1]} k={P.shape[0]} L={L} Q={Y.shape[0]}")
    h = B.os_ann_build_proj(dev(X), L, dev(P), None if mu is None else dev(mu))
    o = orc.build_index_proj(X, L, mu, P)
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
        for budget in budgets:
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget)
            torch.cuda.synchronize()
            oi, od32, od64, on = orc.search_proj(X, o, Y, budget)
            assert np.array_equal(gn.cpu().numpy(), on), (tag, budget)
            assert np.array_equal(gi.cpu().numpy(), oi), (tag, budget)
            assert np.array_equal(gd.cpu().numpy().view(np.uint32), od32.view(np.uint32)), (tag, budget)
            # the screened search walks the keys and screens the full vectors
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget, mode=B.OS_ANN_MODE_TILED)
            torch.cuda.synchronize()
            check_screened(orc, X, Y, (gi.cpu().numpy(), gd.cpu().numpy(), gn.cpu().numpy()),
                           orc.search_tiled(X, o, Y, budget, R=8), (tag, "tiled", budget))
    finally:
        B.os_ann_free(h)


def test_keyed_gaussian(orc):
    X = _scaled_gauss(6000, 24, 5103)
    Y = _scaled_gauss(300, 24, 5104)
    mu, P, _ = orc.pca_basis(X, 8)
    check_proj(orc, X, Y, 2, mu, P, (1, 60, 700, 5000, 10 ** 9), "gauss d24 k8")
    check_proj(orc, X, Y, 3, None, P, (40, 900), "gauss d24 k8 no centring")


def test_keyed_identity_equals_plain_table(orc):
    X = W.gaussian_db(5000, 12, seed=5105)
    Y = W.gaussian_queries(150, 12, seed=5106)
    h1 = B.os_ann_build_ex(dev(X), 2)
    hp = B.os_ann_build_proj(dev(X), 2, dev(np.eye(12, dtype=np.float32)))
    try:
        for budget in (1, 100, 2000):
            a = B.os_ann_search_ex(h1, dev(Y), budget)
            b = B.os_ann_search_ex(hp, dev(Y), budget)
            torch.cuda.synchronize()
            for u, v in zip(a, b):
                assert torch.equal(u, v)
    finally:
        B.os_ann_free(h1)
        B.os_ann_free(hp)


def test_keyed_descriptor_u8_and_patches_f16(orc):
    X = W.descriptor_db(12000, 128, seed=5107)
    Y, _ = W.descriptor_queries(X, 200)
    mu, P, _ = orc.pca_basis(X, 16)
    check_proj(orc, X, Y, 2, mu, P, (50, 600, 4000), "desc u8 k16")
    img = W.patch_field(128)
    Xp = W.patch_rows(img)
    Yimg = np.roll(img, (3, 5), axis=(0, 1)) + np.random.default_rng(11).normal(0, 0.05, img.shape)
    Yp = W.patch_rows(Yimg)[::53]
    mu, P, _ = orc.pca_basis(Xp, 16)
    check_proj(orc, Xp, Yp, 2, mu, P, (30, 800), "patches f16 k16")


def test_keyed_errors():
    X = W.gaussian_db(500, 8, seed=5108)
    P = dev(np.eye(8, dtype=np.float32)[:4])
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_proj(dev(X), 5, P)  # L > k
    assert e.value.code == B.OS_ANN_EINVAL
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_pca(dev(X), 9)
    assert e.value.code == B.OS_ANN_EINVAL
    h = B.os_ann_build_proj(dev(X), 2, P)
    try:
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_classify(h, dev(W.gaussian_queries(3, 8, seed=1)), 10)
        assert e.value.code == B.OS_ANN_ENOTSUP
        i, d, n = B.os_ann_search_ex(h, dev(np.zeros((0, 8), dtype=np.float32)), 10)
        assert i.numel() == 0
    finally:
        B.os_ann_free(h)
