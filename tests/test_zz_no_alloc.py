"""os_ann_search_static: the FP32 search with the library's fixed device
scratch (no allocation) gives what os_ann_search_ex gives, bit for bit, on
two calls in a row (the second with fewer queries), for row budgets and
fixed-C walks, FP32 and uint8 tables; batches beyond the scratch, tiled
mode and workspaces are rejected on the host."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()


def _static(h, yq, budget, cones=False):
    Q = yq.shape[0]
    oi = torch.full((Q,), -7, dtype=torch.int64, device="cuda")
    od = torch.full((Q,), -1.0, dtype=torch.float32, device="cuda")
    on = torch.full((Q,), -1, dtype=torch.int64, device="cuda")
    B.os_ann_search_static(h, yq, budget, oi, od, on, cones=cones)
    torch.cuda.synchronize()
    return oi.cpu().numpy(), od.cpu().numpy(), on.cpu().numpy()


def _ex(h, yq, budget, cones=False):
    i, d, n = B.os_ann_search_ex(h, yq, budget, cones=cones)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy(), n.cpu().numpy()


def _same(a, b, tag):
    assert np.array_equal(a[0], b[0]), tag
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32)), tag
    assert np.array_equal(a[2], b[2]), tag


@pytest.mark.parametrize("kind", ["gauss", "desc"])
def test_static_matches_search_ex(orc, kind):
    if kind == "gauss":
        X = W.gaussian_db(50000, 64, seed=9101)
        Y1 = W.gaussian_queries(3000, 64, seed=9102)
        Y2 = W.gaussian_queries(700, 64, seed=9103)
    else:
        X = W.descriptor_db(30000, 128, seed=9104)
        Y1, _ = W.descriptor_queries(X, 2000)
        Y2 = Y1[::7].copy() + 1.0
    h = B.os_ann_build_ex(dev(X), 2)
    try:
        for budget, cones in ((1500, False), (12, True)):
            for Y in (Y1, Y2):  # two calls in a row, the second smaller
                say(f"[static] {kind} Q={len(Y)} budget={budget} cones={cones}")
                yq = dev(Y)
                got = _static(h, yq, budget, cones)
                _same(got, _ex(h, yq, budget, cones), (kind, len(Y), budget, cones))
                if not cones:
                    oi, od32, od64, on = orc.search(X, orc.build_index(X, 2), Y, budget)
                    assert np.array_equal(got[0], oi) and np.array_equal(got[2], on)
    finally:
        B.os_ann_free(h)


def test_static_rejections():
    X = W.gaussian_db(5000, 64, seed=9201)
    h = B.os_ann_build_ex(dev(X), 2)
    try:
        big = torch.zeros(200_000, 64, dtype=torch.float32, device="cuda")
        oi = torch.empty(200_000, dtype=torch.int64, device="cuda")
        od = torch.empty(200_000, dtype=torch.float32, device="cuda")
        with pytest.raises(B.OsAnnError) as e:
            B.os_ann_search_static(h, big, 100, oi, od)
        assert e.value.code == B.OS_ANN_EINVAL and "split the batch" in str(e.value)
        small = dev(W.gaussian_queries(10, 64, seed=9202))
        o = B.os_ann_search_opts(B.OS_ANN_MODE_TILED, 8, B.OS_ANN_F32, 0, 0, None, 0)
        rc = B.lib().os_ann_search_static(h, small.data_ptr(), 10, 100, o, oi.data_ptr(), od.data_ptr(), None)
        assert rc == B.OS_ANN_ENOTSUP
        ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        o = B.os_ann_search_opts(B.OS_ANN_MODE_FP32, 8, B.OS_ANN_F32, 0, 0, ws.data_ptr(), 1 << 20)
        rc = B.lib().os_ann_search_static(h, small.data_ptr(), 10, 100, o, oi.data_ptr(), od.data_ptr(), None)
        assert rc == B.OS_ANN_EINVAL
        o = B.os_ann_search_opts(B.OS_ANN_MODE_FP32, 8, B.OS_ANN_F32, B.OS_ANN_FLAG_GRAPH, 0, None, 0)
        rc = B.lib().os_ann_search_static(h, small.data_ptr(), 10, 100, o, oi.data_ptr(), od.data_ptr(), None)
        assert rc == B.OS_ANN_EINVAL
        torch.cuda.synchronize()
    finally:
        B.os_ann_free(h)
