"""GPU parity of the structured bases (Section 3.D; reading R14: basis
H diag(s) by the fast Walsh-Hadamard transform in FP32, unnormalised)
against the oracle through the C ABI.  Per basis: cones, packed top-L
pairs, offsets and permutation bit-exact (both sides run the butterflies in
the same order, each a + b and a - b rounded in FP32).  Searches (row
budget and fixed C): result rows, FP32 distances and distinct-row counts
bit-exact."""
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


def signs(R, K, seed):
    return np.where(np.random.default_rng(seed).random((R, K)) < 0.5, -1.0, 1.0).astype(np.float32)


def check_wht(orc, X, Y, L, sg, budgets, tag, cones=()):
    say(f"[wht] {tag} N={X.shape[0]} D={X.shape[1]} L={L} R={len(sg)} Q={Y.shape[0]} dtype={X.dtype}")
    h = B.os_ann_build_wht(dev(X), L, dev(sg))
    o = orc.build_index_wht(X, L, sg)
    try:
        for r in range(len(sg)):
            ex = B.os_ann_export_basis(h, r)
            torch.cuda.synchronize()
            t = o["tables"][r]
            assert np.array_equal(ex["cone"].cpu().numpy().view(np.uint32).astype(np.int64), t["cone"]), (tag, r)
            ti, ts = unpack_top(ex["top"].cpu().numpy().view(np.uint64), L)
            assert np.array_equal(ti, t["top"]) and np.array_equal(ts, t["sign"]), (tag, r)
            assert np.array_equal(ex["offsets"].cpu().numpy(), t["offsets"]), (tag, r)
            assert np.array_equal(ex["perm"].cpu().numpy(), t["perm"]), (tag, r)
        yq = dev(Y)
        for budget, c in [(b, False) for b in budgets] + [(b, True) for b in cones]:
            say(f"[wht] {tag} budget={budget} cones={c}")
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget, cones=c)
            torch.cuda.synchronize()
            gi, gd, gn = gi.cpu().numpy(), gd.cpu().numpy(), gn.cpu().numpy()
            oi, od32, od64, on = orc.search_rot(X, o, Y, budget, cones=c)
            assert np.array_equal(gn, on), (tag, budget, c)
            assert np.array_equal(gi, oi), (tag, budget, c)
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), (tag, budget, c)
    finally:
        B.os_ann_free(h)


@pytest.mark.parametrize("D", [16, 64, 128, 256])
def test_wht_gaussian(orc, D):
    X = W.gaussian_db(12000, D, seed=8101 + D)
    Y = W.gaussian_queries(203, D, seed=8102 + D)
    check_wht(orc, X, Y, 2, signs(3, D, 8103 + D), (1, 300, 5000), f"gauss d{D}", cones=(1, 20))


def test_wht_descriptor_u8_and_patches_f16(orc):
    X = W.descriptor_db(8000, 128)
    Y, _ = W.descriptor_queries(X, 150)
    check_wht(orc, X, Y, 2, signs(2, 128, 8110), (64, 2000), "desc u8 R2")
    img = W.patch_field(96)
    Xp = W.patch_rows(img)
    Yp = W.patch_rows(np.roll(img, (1, 2), axis=(0, 1)))[::31]
    check_wht(orc, Xp, Yp, 2, signs(4, 64, 8111), (100, 1500), "patches f16 R4", cones=(3,))


def test_wht_errors():
    X = W.gaussian_db(500, 24, seed=8112)
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_wht(dev(X), 2, dev(signs(2, 24, 8113)))  # D not a power of two
    assert e.value.code == B.OS_ANN_EINVAL
    X = W.gaussian_db(500, 16, seed=8114)
    bad = signs(2, 16, 8115)
    bad[1, 3] = 0.5
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_wht(dev(X), 2, dev(bad))
    assert e.value.code == B.OS_ANN_EINVAL
    h = B.os_ann_build_wht(dev(X), 2, dev(signs(2, 16, 8116)))
    try:
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_search_ex(h, dev(W.gaussian_queries(3, 16, seed=1)), 10, mode=B.OS_ANN_MODE_TILED)
        assert e.value.code == B.OS_ANN_ENOTSUP
    finally:
        B.os_ann_free(h)
