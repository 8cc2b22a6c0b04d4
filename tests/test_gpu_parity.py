"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Keys, buckets and candidate counts must be bit-exact;
FP32 distances must equal the oracle's term-by-term FP32 value bit for bit
and lie within 1e-5 relative of its double value; result rows must match."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import dev, gpu_index, gpu_search, say, unpack_top

pytestmark = pytest.mark.gpu

RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


def check_index(orc, X, L, tag):
    say(f"[index] {tag} N={X.shape[0]} D={X.shape[1]} L={L} dtype={X.dtype}")
    h, g = gpu_index(X, L)
    o = orc.build_index(X, L)
    assert np.array_equal(g["cone"], o["cone"]), tag
    assert np.array_equal(g["top_idx"], o["top"]), tag
    assert np.array_equal(g["top_sign"], o["sign"]), tag
    assert np.array_equal(g["offsets"], o["offsets"]), tag
    assert np.array_equal(g["perm"], o["perm"]), tag
    rows = B.os_ann_export_rows(h).cpu().numpy()
    assert np.array_equal(rows, X[o["perm"]].astype(np.float32)), tag
    info = B.os_ann_info(h)
    assert info["n_nonempty"] == int((np.diff(o["offsets"]) > 0).sum())
    return h, o


def check_search(orc, X, o, h, Y, budget, tag):
    say(f"[search] {tag} Q={Y.shape[0]} B={budget}")
    gi, gd, gn = gpu_search(h, Y, budget)
    oi, od32, od64, on = orc.search(X, o, Y, budget)
    assert np.array_equal(gn, on), tag
    assert np.array_equal(gi, oi), tag
    assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), tag
    rel = np.abs(gd.astype(np.float64) - od64) / np.maximum(od64, 1e-300)
    assert (rel <= RTOL).all(), (tag, rel.max())


def test_fig2_toy_dataset(orc):
    X = np.array([[-22, 12, 5], [-21, -19, -12], [29, 24, -13], [44, 17, -4], [49, -6, 5], [57, 8, -2],
                  [-3, -18, 10], [-1, -13, 0], [5, 11, 4], [11, 14, -3], [14, 25, 23], [-36, 23, -47],
                  [5, 26, -27], [9, -2, -17], [12, 5, -14], [-7, 11, 22]], dtype=np.float32)
    for L in (1, 2, 3):
        h, o = check_index(orc, X, L, f"fig2 L={L}")
        Y = X[::3] + np.float32(0.5)
        for budget in (1, 3, 16):
            check_search(orc, X, o, h, Y, budget, f"fig2 L={L}")
        B.os_ann_free(h)


@pytest.mark.parametrize("dtype", [np.float32, np.float16, np.uint8])
@pytest.mark.parametrize("D,L", [(1, 1), (3, 2), (5, 3), (13, 2), (16, 1), (33, 4), (64, 2), (12, 7),
                                 (128, 2), (256, 2)])
def test_keys_and_buckets_ties(orc, D, L, dtype):
    """Tie-heavy small integers (and -0.0 for float types), ragged D."""
    if dtype == np.uint8:
        X = W.tie_heavy(3001, D, seed=D * 10 + L, values=(0, 1, 2, 3)).astype(np.uint8)
    else:
        X = W.tie_heavy(3001, D, seed=D * 10 + L).astype(dtype)
    h, o = check_index(orc, X, L, f"ties D={D} L={L}")
    B.os_ann_free(h)


@pytest.mark.parametrize("D,L,N", [(16, 1, 16384), (64, 2, 70001), (8, 3, 5000), (20, 4, 9000)])
def test_search_gaussian(orc, D, L, N):
    X = W.gaussian_db(N, D, seed=500 + D)
    Y = W.gaussian_queries(700, D, seed=600 + D)
    h, o = check_index(orc, X, L, f"gauss D={D} L={L}")
    for budget in (1, 100, 512, 3000, 9000, N // 2, N, 10 * N):
        check_search(orc, X, o, h, Y, budget, f"gauss D={D} L={L}")
    B.os_ann_free(h)


def test_search_tie_heavy_distances(orc):
    """Integer data: many equal distances, ties go to the lower row."""
    X = W.tie_heavy(5000, 12, seed=77)
    Y = W.tie_heavy(400, 12, seed=78)
    h, o = check_index(orc, X, 2, "tie search")
    for budget in (1, 50, 700, 5000):
        check_search(orc, X, o, h, Y, budget, "tie search")
    B.os_ann_free(h)


def test_descriptor_uint8(orc):
    X = W.descriptor_db(30000, 128, seed=W.SEEDS["desc_db"])
    Y, src = W.descriptor_queries(X, 300)
    h, o = check_index(orc, X, 2, "descriptor u8")
    for budget in (256, 1024, 4096):
        check_search(orc, X, o, h, Y, budget, "descriptor u8")
    B.os_ann_free(h)


def test_patches_fp16(orc):
    img = W.patch_field(256)
    X = W.patch_rows(img)
    Yimg = np.roll(img, (3, 5), axis=(0, 1)) + np.random.default_rng(9).normal(0, 0.05, img.shape)
    Y = W.patch_rows(Yimg)[::97]
    h, o = check_index(orc, X, 2, "patches f16")
    for budget in (64, 1024):
        check_search(orc, X, o, h, Y, budget, "patches f16")
    B.os_ann_free(h)


def test_classify_matches_oracle(orc):
    X = W.gaussian_db(40000, 32, seed=801)
    Y = W.gaussian_queries(500, 32, seed=802)
    Y[0, :] = 0.0
    Y[1, 3] = -0.0
    h, o = check_index(orc, X, 3, "classify")
    top, sg, cone = orc.hash_rows(Y, 3)
    for budget in (1, 777, 39999):
        say(f"[classify] B={budget}")
        c, t, n = B.os_ann_classify(h, dev(Y), budget)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint32), cone.astype(np.uint32))
        ti, ts = unpack_top(t.cpu().numpy().view(np.uint64), 3)
        assert np.array_equal(ti, top) and np.array_equal(ts, sg)
        want = [orc.probe(y, 3, o["offsets"], budget)[1] for y in Y]
        assert n.cpu().numpy().tolist() == want
    B.os_ann_free(h)


def test_edge_cases(orc):
    say("[edge] N=1")
    X = np.array([[0.5, -2.0, 1.0]], dtype=np.float32)
    h, o = check_index(orc, X, 2, "N=1")
    check_search(orc, X, o, h, W.gaussian_queries(5, 3, seed=1), 1, "N=1")
    say("[edge] Q=0")
    i, d, n = B.os_ann_search_ex(h, dev(np.zeros((0, 3), np.float32)), 5)
    assert i.numel() == 0
    B.os_ann_free(h)
    say("[edge] identical rows")
    X = np.ones((3000, 8), dtype=np.float32)
    h, o = check_index(orc, X, 2, "identical")
    check_search(orc, X, o, h, W.gaussian_queries(50, 8, seed=2), 10, "identical")
    B.os_ann_free(h)
    say("[edge] errors")
    bad = W.gaussian_db(100, 8, seed=3)
    bad[7, 2] = np.nan
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_ex(dev(bad), 2)
    assert e.value.code == B.OS_ANN_ENONFINITE
    bad[7, 2] = np.inf
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_ex(dev(bad.astype(np.float16)), 2)
    assert e.value.code == B.OS_ANN_ENONFINITE
    # with the low-precision copy the table's check is taken at the copy's end
    for dt in (np.float32, np.float16):
        bad[7, 2] = np.nan if dt == np.float32 else np.inf
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_build_ex(dev(bad.astype(dt)), 2, want_lowp=True)
        assert e.value.code == B.OS_ANN_ENONFINITE
    # C(256,7) 2^7 = 1.7e15 cones: a sparse table (reading R15) of 10 rows
    Xs = W.gaussian_db(10, 256, seed=4)
    Ys = W.gaussian_queries(3, 256, seed=5)
    hs = B.os_ann_build_ex(dev(Xs), 7)
    try:
        info = B.os_ann_info(hs)
        assert info["n_cones"] == orc.num_cones(256, 7) and 1 <= info["n_nonempty"] <= 10
        os_ = orc.build_index_sparse(Xs, 7)
        for budget, cones in ((10, False), (1, True)):
            gi, gd, gn = B.os_ann_search_ex(hs, dev(Ys), budget, cones=cones)
            torch.cuda.synchronize()
            oi, od32, od64, on = orc.search_sparse(Xs, os_, Ys, budget, cones=cones)
            assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gn.cpu().numpy(), on)
            assert np.array_equal(gd.cpu().numpy().view(np.uint32), od32.view(np.uint32))
    finally:
        B.os_ann_free(hs)
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_build_ex(dev(W.gaussian_db(10, 4, seed=4)), 5)
    assert e.value.code == B.OS_ANN_EINVAL
    h = B.os_ann_build_ex(dev(W.gaussian_db(100, 4, seed=5)), 1)
    with pytest.raises(B.OsAnnError) as e:
        B.os_ann_search_ex(h, dev(W.gaussian_queries(3, 4, seed=6)), 0)
    assert e.value.code == B.OS_ANN_EINVAL
    B.os_ann_free(h)


def test_db_freed_after_build(orc):
    X = W.gaussian_db(20000, 16, seed=901)
    Y = W.gaussian_queries(200, 16, seed=902)
    t = dev(X)
    h = B.os_ann_build_ex(t, 1)
    del t
    torch.cuda.empty_cache()
    junk = torch.full((20000 * 16,), 7.0, device="cuda")  # reuse the freed memory
    o = orc.build_index(X, 1)
    check_search(orc, X, o, h, Y, 512, "db freed")
    del junk
    B.os_ann_free(h)


def test_batch_invariance_and_determinism(orc):
    X = W.gaussian_db(50000, 32, seed=911)
    Y = W.gaussian_queries(300, 32, seed=912)
    h = B.os_ann_build_ex(dev(X), 2)
    full = gpu_search(h, Y, 2000)
    again = gpu_search(h, Y, 2000)
    for a, b in zip(full, again):
        assert np.array_equal(a, b)
    for s, e in ((0, 1), (5, 6), (17, 150), (150, 300)):
        part = gpu_search(h, Y[s:e], 2000)
        for a, b in zip(full, part):
            assert np.array_equal(a[s:e], b)
    h2 = B.os_ann_build_ex(dev(X), 2)
    e1, e2 = B.os_ann_export(h), B.os_ann_export(h2)
    for k in e1:
        assert torch.equal(e1[k], e2[k])
    B.os_ann_free(h)
    B.os_ann_free(h2)


def test_two_streams_with_workspaces(orc):
    X = W.gaussian_db(60000, 64, seed=921)
    Y = W.gaussian_queries(2000, 64, seed=922)
    h = B.os_ann_build_ex(dev(X), 2)
    ref = gpu_search(h, Y, 1024)
    yd = dev(Y)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    nb = B.os_ann_workspace_bytes(h, 1000, 1024)
    w1 = torch.empty(nb, dtype=torch.uint8, device="cuda")
    w2 = torch.empty(nb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    a = B.os_ann_search_ex(h, yd[:1000], 1024, stream=s1, workspace=w1)
    b = B.os_ann_search_ex(h, yd[1000:], 1024, stream=s2, workspace=w2)
    torch.cuda.synchronize()
    for k in range(3):
        got = np.concatenate([a[k].cpu().numpy(), b[k].cpu().numpy()])
        assert np.array_equal(got, ref[k])
    B.os_ann_free(h)
