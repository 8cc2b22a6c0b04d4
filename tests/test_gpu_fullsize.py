"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (the whole query batch in one call), on sampled queries the
oracle recomputes one by one.

* 1e6 x 64 i.i.d. Gaussian FP32, L=2, 1e4 queries: budgets 256/1024/4096 and
  327680 (the smallest swept budget at which recall@1 reaches 0.9), both modes.
* 1e6 x 128 descriptor-like uint8 rows, L=2, 1e4 noisy queries, both modes.
* ~4.2e6 mean-removed 8x8 FP16 patches of a 2048x2048 1/f field, L=2, queries
  are all patches of the shifted noisy field (~4.2e6), tiled mode.
* the 1e6 x 64 Gaussian workload with four bases (Section 3.A).
* the descriptor workload through the PCA front-end (Section 4.B), k = 16.
* the Gaussian workload in fixed-C mode (C = 16, 512, 2048 cones), both modes.
* the Gaussian workload as a sparse table (L = 5, 2.4e8 cones) and with four
  structured (Walsh-Hadamard) bases.

The index itself (every key, bucket offset and permutation entry) is compared
in full; searches are compared on a spread sample of queries."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import candidates_of, check_screened, dev, say, unpack_top

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


def full_index(orc, X, L, tag):
    say(f"[full] {tag}: building N={X.shape[0]} D={X.shape[1]} L={L} dtype={X.dtype}")
    h = B.os_ann_build_ex(dev(X), L, want_lowp=True)
    ex = B.os_ann_export(h)
    torch.cuda.synchronize()
    o = orc.build_index(X, L)
    cone = ex["cone"].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(cone, o["cone"]), tag
    ti, ts = unpack_top(ex["top"].cpu().numpy().view(np.uint64), L)
    assert np.array_equal(ti, o["top"]) and np.array_equal(ts, o["sign"]), tag
    assert np.array_equal(ex["offsets"].cpu().numpy(), o["offsets"]), tag
    assert np.array_equal(ex["perm"].cpu().numpy(), o["perm"]), tag
    del ex
    return h, o


def sample_ids(Q, n):
    return np.unique(np.linspace(0, Q - 1, n).astype(np.int64))


def fp32_sampled(orc, X, o, h, Y, yq, budget, sample, tag, cones=False):
    say(f"[full] {tag}: fp32 Q={Y.shape[0]} B={budget} cones={cones}")
    gi, gd, gn = B.os_ann_search_ex(h, yq, budget, mode=B.OS_ANN_MODE_FP32, cones=cones)
    torch.cuda.synchronize()
    gi, gd, gn = gi.cpu().numpy()[sample], gd.cpu().numpy()[sample], gn.cpu().numpy()[sample]
    oi, od32, od64, on = orc.search(X, o, Y[sample], budget, cones=cones)
    assert np.array_equal(gn, on), tag
    assert np.array_equal(gi, oi), tag
    assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), tag
    assert (np.abs(gd - od64) <= RTOL * np.maximum(od64, 1e-300)).all(), tag


def tiled_sampled(orc, X, o, h, Y, yq, budget, sample, tag, R=8, max_mismatch=0.02, cones=False):
    say(f"[full] {tag}: tiled Q={Y.shape[0]} B={budget} cones={cones} sample={len(sample)}")
    gi, gd, gn = B.os_ann_search_ex(h, yq, budget, mode=B.OS_ANN_MODE_TILED, rerank_r=R, cones=cones)
    torch.cuda.synchronize()
    gi, gd, gn = gi.cpu().numpy()[sample], gd.cpu().numpy()[sample], gn.cpu().numpy()[sample]
    Ys = Y[sample]
    ot = orc.search_tiled(X, o, Ys, budget, R=R, cones=cones)
    check_screened(orc, X, Ys, (gi, gd, gn), ot, (tag, "tiled", budget), max_mismatch=max_mismatch,
                   is_candidate=candidates_of(orc, o, Ys, budget, cones=cones))


@pytest.fixture(scope="module")
def gauss1m(orc):
    X = W.gaussian_db(1_000_000, 64, W.SEEDS["gauss64_db"])
    Y = W.gaussian_queries(10_000, 64, W.SEEDS["gauss64_q"])
    h, o = full_index(orc, X, 2, "gauss 1e6x64")
    yield X, Y, h, o, dev(Y)
    B.os_ann_free(h)


HEADLINE_BUDGET = 327680  # smallest swept budget at which recall@1 reaches 0.9 (both modes)


def test_gaussian_1m_d64(orc, gauss1m):
    X, Y, h, o, yq = gauss1m
    for budget, n in ((256, 400), (1024, 400), (4096, 200)):
        s = sample_ids(len(Y), n)
        fp32_sampled(orc, X, o, h, Y, yq, budget, s, "gauss 1e6x64")
        tiled_sampled(orc, X, o, h, Y, yq, budget, s, "gauss 1e6x64")
    # fixed-C mode (Section 3, Table III) in the same launch shape
    for C, n in ((16, 300), (512, 100), (2048, 48)):
        s = sample_ids(len(Y), n)
        fp32_sampled(orc, X, o, h, Y, yq, C, s, "gauss 1e6x64", cones=True)
        tiled_sampled(orc, X, o, h, Y, yq, C, s, "gauss 1e6x64", cones=True)


@pytest.mark.timeout(900)  # the oracle's FP32 search of 10,000 queries takes a minute or two
def test_gaussian_1m_d64_headline_all_queries(orc, gauss1m):
    # the benchmark's configuration in full: candidate counts of both modes
    # for every query against the oracle's walk alone (no distances), then
    # FP32-mode rows and distances for every query against the oracle
    X, Y, h, o, yq = gauss1m
    B_ = HEADLINE_BUDGET
    say(f"[full] headline: oracle candidate counts of all {len(Y)} queries")
    on = np.array([orc.probe(Y[q], 2, o["offsets"], B_)[1] for q in range(len(Y))], dtype=np.int64)
    for mode in (B.OS_ANN_MODE_TILED, B.OS_ANN_MODE_FP32):
        say(f"[full] headline: GPU mode {mode} B={B_}")
        gi, gd, gn = B.os_ann_search_ex(h, yq, B_, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(gn.cpu().numpy(), on), mode
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    parts = []
    for q0 in range(0, len(Y), 2500):  # in parts, so that progress shows
        parts.append(orc.search(X, o, Y[q0:q0 + 2500], B_))
        say(f"[full] headline: oracle FP32 search, {q0 + len(parts[-1][0])} of {len(Y)} queries")
    oi, od32, od64, on2 = (np.concatenate(c) for c in zip(*parts))
    assert np.array_equal(on2, on)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32))
    rel = np.abs(gd - od64) / np.maximum(od64, 1e-300)
    say(f"[full] headline: FP32 rows and distances equal for all {len(Y)} queries; "
        f"max rel err vs FP64 {rel.max():.2e}")
    assert (rel <= RTOL).all()


@pytest.mark.timeout(600)
def test_gaussian_1m_d64_headline_tiled(orc, gauss1m):
    # the tiled mode at the benchmark's configuration on 1,000 spread queries
    X, Y, h, o, yq = gauss1m
    tiled_sampled(orc, X, o, h, Y, yq, HEADLINE_BUDGET, sample_ids(len(Y), 1000), "gauss 1e6x64 headline")


def test_descriptor_1m_d128_u8(orc):
    X = W.descriptor_db(1_000_000, 128)
    Y, _ = W.descriptor_queries(X, 10_000)
    h, o = full_index(orc, X, 2, "desc 1e6x128 u8")
    yq = dev(Y)
    try:
        for budget, n in ((256, 300), (1024, 300), (4096, 150)):
            s = sample_ids(len(Y), n)
            fp32_sampled(orc, X, o, h, Y, yq, budget, s, "desc 1e6x128 u8")
            tiled_sampled(orc, X, o, h, Y, yq, budget, s, "desc 1e6x128 u8")
    finally:
        B.os_ann_free(h)


def test_patches_4m_fp16(orc):
    X, Y = W.patch_pair(2048)
    h, o = full_index(orc, X, 2, "patches 2048^2 f16")
    yq = dev(Y)
    try:
        for budget, n in ((64, 300), (1024, 200)):
            tiled_sampled(orc, X, o, h, Y, yq, budget, sample_ids(len(Y), n), "patches 2048^2 f16")
        fp32_sampled(orc, X, o, h, Y, yq, 1024, sample_ids(len(Y), 200), "patches 2048^2 f16")
    finally:
        B.os_ann_free(h)


def test_several_bases_1m_d64(orc):
    # four bases (the first the identity) on the full 1e6 x 64 workload, at the
    # budget where recall@1 reaches 0.9, in the benchmark's launch shape
    X = W.gaussian_db(1_000_000, 64, W.SEEDS["gauss64_db"])
    Y = W.gaussian_queries(10_000, 64, W.SEEDS["gauss64_q"])
    rots = W.random_bases(4, 64)
    say("[full] several bases: building 4 tables")
    h = B.os_ann_build_rot(dev(X), 2, dev(rots))
    o = orc.build_index_rot(X, 2, rots)
    try:
        for r in range(4):
            ex = B.os_ann_export_basis(h, r)
            torch.cuda.synchronize()
            assert np.array_equal(ex["offsets"].cpu().numpy(), o["tables"][r]["offsets"]), r
            assert np.array_equal(ex["perm"].cpu().numpy(), o["tables"][r]["perm"]), r
            del ex
        yq = dev(Y)
        for budget, n in ((4096, 200), (131072, 40)):
            s = sample_ids(len(Y), n)
            say(f"[full] several bases: budget {budget}")
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget)
            torch.cuda.synchronize()
            gi, gd, gn = gi.cpu().numpy()[s], gd.cpu().numpy()[s], gn.cpu().numpy()[s]
            oi, od32, od64, on = orc.search_rot(X, o, Y[s], budget)
            assert np.array_equal(gn, on) and np.array_equal(gi, oi), budget
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), budget
    finally:
        B.os_ann_free(h)


def test_descriptor_1m_pca16(orc):
    # the PCA front-end at the full descriptor size: axes against the
    # oracle's, then the keyed table (with the oracle's axes on both sides)
    # compared in full and searched in the benchmark's launch shape
    X = W.descriptor_db(1_000_000, 128)
    Y, _ = W.descriptor_queries(X, 10_000)
    say("[full] pca: axes of 1e6 x 128 u8")
    mu, P, var = B.os_ann_pca(dev(X), 16)
    omu, oP, ovar = orc.pca_basis(X, 16)
    assert np.allclose(mu, omu, rtol=1e-6, atol=1e-6)
    assert np.allclose(var, ovar, rtol=1e-9)
    assert np.allclose(P, oP, atol=1e-5)
    say("[full] pca: keyed table")
    h = B.os_ann_build_proj(dev(X), 2, dev(oP), dev(omu))
    o = orc.build_index_proj(X, 2, omu, oP)
    try:
        ex = B.os_ann_export(h)
        torch.cuda.synchronize()
        assert np.array_equal(ex["cone"].cpu().numpy().view(np.uint32).astype(np.int64), o["cone"])
        assert np.array_equal(ex["offsets"].cpu().numpy(), o["offsets"])
        assert np.array_equal(ex["perm"].cpu().numpy(), o["perm"])
        del ex
        yq = dev(Y)
        for budget, n in ((64, 300), (1024, 200)):
            s = sample_ids(len(Y), n)
            say(f"[full] pca: budget {budget}")
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget)
            torch.cuda.synchronize()
            gi, gd, gn = gi.cpu().numpy()[s], gd.cpu().numpy()[s], gn.cpu().numpy()[s]
            oi, od32, od64, on = orc.search_proj(X, o, Y[s], budget)
            assert np.array_equal(gn, on) and np.array_equal(gi, oi), budget
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), budget
    finally:
        B.os_ann_free(h)


def test_sparse_1m_d64_l5(orc):
    # the 1e6 x 64 Gaussian rows as a sparse table (L = 5: 2.4e8 cones), in
    # the benchmark's launch shape: the whole index compared, searches sampled
    X = W.gaussian_db(1_000_000, 64, W.SEEDS["gauss64_db"])
    Y = W.gaussian_queries(10_000, 64, W.SEEDS["gauss64_q"])
    say("[full] sparse L=5: building")
    h = B.os_ann_build_ex(dev(X), 5)
    o = orc.build_index_sparse(X, 5)
    try:
        ex = B.os_ann_export_sparse(h)
        torch.cuda.synchronize()
        assert np.array_equal(ex["cone_ids"].cpu().numpy(), o["keys"])
        assert np.array_equal(ex["offsets"].cpu().numpy(), o["offsets"])
        assert np.array_equal(ex["perm"].cpu().numpy(), o["perm"])
        del ex
        yq = dev(Y)
        for budget, cones, n in ((1024, False, 60), (64, True, 60)):
            s = sample_ids(len(Y), n)
            say(f"[full] sparse L=5: budget {budget} cones={cones}")
            gi, gd, gn = B.os_ann_search_ex(h, yq, budget, cones=cones)
            torch.cuda.synchronize()
            gi, gd, gn = gi.cpu().numpy()[s], gd.cpu().numpy()[s], gn.cpu().numpy()[s]
            oi, od32, od64, on = orc.search_sparse(X, o, Y[s], budget, cones=cones)
            assert np.array_equal(gn, on) and np.array_equal(gi, oi), budget
            assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32)), budget
    finally:
        B.os_ann_free(h)


def test_structured_bases_1m_d64(orc):
    # four Walsh-Hadamard bases on the full workload at the several-bases
    # benchmark budget
    X = W.gaussian_db(1_000_000, 64, W.SEEDS["gauss64_db"])
    Y = W.gaussian_queries(10_000, 64, W.SEEDS["gauss64_q"])
    sg = W.random_signs(4, 64)
    say("[full] structured bases: building 4 tables")
    h = B.os_ann_build_wht(dev(X), 2, dev(sg))
    o = orc.build_index_wht(X, 2, sg)
    try:
        for r in range(4):
            ex = B.os_ann_export_basis(h, r)
            torch.cuda.synchronize()
            assert np.array_equal(ex["offsets"].cpu().numpy(), o["tables"][r]["offsets"]), r
            assert np.array_equal(ex["perm"].cpu().numpy(), o["tables"][r]["perm"]), r
            del ex
        s = sample_ids(len(Y), 40)
        gi, gd, gn = B.os_ann_search_ex(h, dev(Y), 131072)
        torch.cuda.synchronize()
        gi, gd, gn = gi.cpu().numpy()[s], gd.cpu().numpy()[s], gn.cpu().numpy()[s]
        oi, od32, od64, on = orc.search_rot(X, o, Y[s], 131072)
        assert np.array_equal(gn, on) and np.array_equal(gi, oi)
        assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32))
    finally:
        B.os_ann_free(h)
