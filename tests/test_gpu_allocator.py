"""Device memory from the caller's allocator (os_ann_set_allocator) and the
plain entry points os_ann_build / os_ann_search.

* Every block the library asks for comes from the hook and goes back to it:
  after os_ann_free nothing the hook handed out is still held.
* A hook that returns NULL part-way through a build or a search makes the
  call fail with OS_ANN_ENOMEM, every block obtained so far is returned (the
  count of live blocks is back where it was), and an index built before
  stays searchable with unchanged results.
* os_ann_build / os_ann_search (FP32 rows, index scratch, null stream) give
  the oracle's rows, FP32 distances bit for bit, and work with PyTorch's
  caching allocator as the hook."""
import numpy as np
import pytest
import torch

from paper_1509_03453_amd import binding as B
from paper_1509_03453_amd import workloads as W
from tests.gpu_util import candidates_of, check_screened, dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    B.os_ann_set_allocator(None, None)


class CountingHook:
    """Blocks from PyTorch tensors; refuses every call from `fail_from` on."""

    def __init__(self):
        self.live = {}
        self.calls = 0
        self.fail_from = None

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.fail_from is not None and self.calls >= self.fail_from:
            return 0
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def free(self, ptr, stream):
        del self.live[ptr]


def _search(h, Y, budget, mode=B.OS_ANN_MODE_FP32):
    i, d, n = B.os_ann_search_ex(h, dev(Y), budget, mode=mode)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy(), n.cpu().numpy()


def test_plain_build_and_search_match_oracle(orc):
    # the plain signatures: os_ann_build(db, N, D, L) and
    # os_ann_search(index, queries, Q, max_candidates, out_idx, out_dist)
    X = W.gaussian_db(40000, 32, seed=8101)
    Y = W.gaussian_queries(777, 32, seed=8102)
    o = orc.build_index(X, 2)
    for hooked in (False, True):
        if hooked:
            B.use_torch_allocator()
        say(f"[alloc] plain build/search, torch allocator={hooked}")
        h = B.os_ann_build(dev(X), 2)
        try:
            for budget in (1, 600, 5000, 40000):
                gi, gd = B.os_ann_search(h, dev(Y), budget)
                torch.cuda.synchronize()
                oi, od32, od64, on = orc.search(X, o, Y, budget)
                assert np.array_equal(gi.cpu().numpy(), oi), budget
                assert np.array_equal(gd.cpu().numpy().view(np.uint32), od32.view(np.uint32)), budget
        finally:
            B.os_ann_free(h)
        B.os_ann_set_allocator(None, None)


def test_hook_owns_every_block_and_enomem_leaks_nothing(orc):
    X = W.gaussian_db(30000, 64, seed=8201)
    Y = W.gaussian_queries(300, 64, seed=8202)
    hook = CountingHook()
    B.os_ann_set_allocator(hook.alloc, hook.free)
    try:
        say("[alloc] index A through the hook")
        ha = B.os_ann_build_ex(dev(X), 2)
        ref = _search(ha, Y, 2000)
        ref_t = _search(ha, Y, 2000, B.OS_ANN_MODE_TILED)  # low-precision copy and scratch from the hook
        held = len(hook.live)
        assert held > 0 and hook.calls >= held
        built = hook.calls
        # a second build refused at each of its first allocations in turn
        Xb = W.gaussian_db(20000, 64, seed=8203)
        for k in range(1, 12):
            hook.fail_from = hook.calls + k
            say(f"[alloc] build B with the hook refusing from its call {k}")
            with pytest.raises(B.OsAnnError) as e:
                B.os_ann_build_ex(dev(Xb), 2)
            assert e.value.code == B.OS_ANN_ENOMEM, e.value
            assert len(hook.live) == held, (k, len(hook.live), held)
        hook.fail_from = None
        # index A is untouched
        for a, b in zip(_search(ha, Y, 2000), ref):
            assert np.array_equal(a, b)
        # a fresh index: its search scratch, then each block of its
        # low-precision copy, refused in turn
        hb = B.os_ann_build_ex(dev(Xb), 2)
        held_b = len(hook.live)
        hook.fail_from = hook.calls + 1
        say("[alloc] FP32 search refused its scratch")
        with pytest.raises(B.OsAnnError) as e:
            _search(hb, Y, 1000)
        assert e.value.code == B.OS_ANN_ENOMEM and len(hook.live) == held_b
        o = orc.build_index(Xb, 2)
        refused = 0
        for k in range(1, 16):
            hook.fail_from = hook.calls + k
            say(f"[alloc] tiled search with the hook refusing from its call {k}")
            try:
                g = _search(hb, Y, 1000, B.OS_ANN_MODE_TILED)
            except B.OsAnnError as err:
                assert err.code == B.OS_ANN_ENOMEM, err
                refused += 1
                # at most the index's own search scratch is kept (freed with the index)
                assert len(hook.live) - held_b in (0, 1), (k, len(hook.live), held_b)
                continue
            break
        assert refused >= 4, refused  # scratch and several blocks of the copy were refused
        hook.fail_from = None
        check_screened(orc, Xb, Y, g, orc.search_tiled(Xb, o, Y, 1000, R=8), "tiled after refusals",
                       is_candidate=candidates_of(orc, o, Y, 1000))
        gi, gd, gn = _search(hb, Y, 1000)
        oi, od32, od64, on = orc.search(Xb, o, Y, 1000)
        assert np.array_equal(gi, oi) and np.array_equal(gn, on)
        assert np.array_equal(gd.view(np.uint32), od32.view(np.uint32))
        B.os_ann_free(hb)
        assert len(hook.live) == held
        for a, b in zip(_search(ha, Y, 2000, B.OS_ANN_MODE_TILED), ref_t):
            assert np.array_equal(a, b)
        B.os_ann_free(ha)
        assert len(hook.live) == 0, len(hook.live)
        assert built > 0
    finally:
        B.os_ann_set_allocator(None, None)
