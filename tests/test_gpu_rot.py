"""GPU parity of the several-bases search (Section 3.A, Algorithm 1) against
the oracle, through the C ABI.  Per basis: cones, packed top-L pairs,
offsets and permutation bit-exact (the coordinates are FP32 term-by-term
products on both sides).  Search: result rows, FP32 distances and the number
of distinct rows analyzed bit-exact; the GPU tells a row's first visit from
its cones in the other bases, the oracle keeps a mark per row."""
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


def check_rot(orc, X, Y, L, rots, budgets, tag, sample=None):
    say(f"[rot] {tag} N={X.shape[0]} D={X.shape[1]} L={L} R={len(rots)} Q={Y.shape[0]} dtype={X.dtype}")
    h = B.os_ann_build_rot(dev(X), L, dev(np.ascontiguousarray(rots, dtype=np.float32)))
    o = orc.build_index_rot(X, L, rots)
    try:
        for r in range(len(rots)):
            ex = B.os_ann_export_basis(h, r)
            torch.cuda.synchronize()
            t = o["tables"][r]
            cone = ex["cone"].cpu().numpy().view(np.uint32).astype(np.int64)
            assert np.array_equal(cone, t["cone"]), (tag, r)
            ti, ts = unpack_top(ex["top"].cpu().numpy().view(np.uint64), L)
            assert np.array_equal(ti, t["top"]) and np.array_equal(ts, t["sign"]), (tag, r)
            assert np.array_equal(ex["offsets"].cpu().numpy(), t["offsets"]), (tag, r)
            assert np.array_equal(ex["perm"].cpu().numpy(), t["perm"]), (tag, r)
        yq = dev(Y)
        s = np.arange(len(Y)) if sample is None else sample
        for budget in budgets:
            say(f"[rot] {tag} budget={budget}")
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget)
            torch.cuda.synchronize()
            gi, gd, gn = gi.cpu().numpy()[s], gd.cpu().numpy()[s], gn.cpu().numpy()[s]
            oi, od32, od64, on = orc.search_rot(X, o, Y[s], budget)
            assert np.array_equal(gn, on), (tag, budget)
            assert np.array_equal(gi, oi), (tag, budget)
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), (tag, budget)
            assert (np.abs(gd - od64) <= 1e-5 * np.maximum(od64, 1e-300)).all(), (tag, budget)
    finally:
        B.os_ann_free(h)


def test_rot_gaussian(orc):
    X = W.gaussian_db(6000, 16, seed=3101)
    Y = W.gaussian_queries(300, 16, seed=3102)
    check_rot(orc, X, Y, 2, W.random_bases(4, 16, seed=3103), (1, 60, 700, 5000, 10 ** 9), "gauss d16 R4")


def test_rot_gaussian_d64_l2(orc):
    X = W.gaussian_db(40000, 64, seed=3104)
    Y = W.gaussian_queries(200, 64, seed=3105)
    check_rot(orc, X, Y, 2, W.random_bases(3, 64, seed=3106), (300, 4000), "gauss d64 R3")


def test_rot_one_identity_basis_equals_single_basis(orc):
    X = W.gaussian_db(5000, 12, seed=3107)
    Y = W.gaussian_queries(150, 12, seed=3108)
    h1 = B.os_ann_build_ex(dev(X), 2)
    hr = B.os_ann_build_rot(dev(X), 2, dev(np.eye(12, dtype=np.float32)[None]))
    try:
        for budget in (1, 100, 2000):
            a = B.os_ann_search_ex(h1, dev(Y), budget)
            b = B.os_ann_search_ex(hr, dev(Y), budget)
            torch.cuda.synchronize()
            for u, v in zip(a, b):
                assert torch.equal(u, v)
    finally:
        B.os_ann_free(h1)
        B.os_ann_free(hr)


def test_rot_ties_and_permutation_bases(orc):
    # permutation bases give exact coordinates; tie-heavy values stress R1/R2
    X = W.tie_heavy(4000, 10, seed=3109)
    Y = W.tie_heavy(120, 10, seed=3110)
    rng = np.random.default_rng(3111)
    rots = np.stack([np.eye(10, dtype=np.float32)[rng.permutation(10)] for _ in range(5)])
    check_rot(orc, X, Y, 3, rots, (10, 300, 3000), "ties perm R5")


def test_rot_descriptor_uint8_and_patches_fp16(orc):
    X = W.descriptor_db(8000, 128, seed=3112)
    Y, _ = W.descriptor_queries(X, 100)
    check_rot(orc, X, Y, 2, W.random_bases(3, 128, seed=3113), (200, 2000), "desc u8 R3")
    img = W.patch_field(128)
    Xp = W.patch_rows(img)
    Yimg = np.roll(img, (3, 5), axis=(0, 1)) + np.random.default_rng(9).normal(0, 0.05, img.shape)
    Yp = W.patch_rows(Yimg)[::61]
    check_rot(orc, Xp, Yp, 2, W.random_bases(2, 64, seed=3114), (100, 1500), "patches f16 R2")


def test_rot_errors():
    X = W.gaussian_db(500, 8, seed=3115)
    rot = dev(W.random_bases(2, 8, seed=3116))
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_rot(dev(X), 2, dev(np.zeros((17, 8, 8), dtype=np.float32)))
    assert e.value.code == B.OS_ANN_EINVAL
    h = B.os_ann_build_rot(dev(X), 2, rot)
    try:
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
