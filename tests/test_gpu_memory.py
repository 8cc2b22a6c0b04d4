"""Device blocks of freed indexes are reused by later builds and searches:
results must not depend on whether a block is fresh, recycled from an index
of the same size or of another size, or fresh again after os_ann_trim."""
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


def _run(X, Y, mode, budget):
    h = B.os_ann_build_ex(dev(X), 2, want_lowp=mode == B.OS_ANN_MODE_TILED)
    try:
        i, d, n = B.os_ann_search_ex(h, dev(Y), budget, mode=mode)
        torch.cuda.synchronize()
        return i.cpu().numpy(), d.cpu().numpy(), n.cpu().numpy()
    finally:
        B.os_ann_free(h)


@pytest.mark.parametrize("mode", [0, 1])
def test_recycled_blocks_give_identical_results(mode):
    X = W.gaussian_db(30000, 32, seed=4101)
    Y = W.gaussian_queries(700, 32, seed=4102)
    Xs = W.gaussian_db(5000, 48, seed=4103)
    Ys = W.gaussian_queries(100, 48, seed=4104)
    say(f"[mem] mode {mode}: fresh, recycled, other sizes, trimmed")
    first = _run(X, Y, mode, 3000)
    again = _run(X, Y, mode, 3000)       # same sizes: every block comes back from the cache
    small = _run(Xs, Ys, mode, 500)      # other sizes in between
    mixed = _run(X, Y, mode, 3000)
    B.os_ann_trim()
    fresh = _run(X, Y, mode, 3000)       # every block from the runtime again
    small2 = _run(Xs, Ys, mode, 500)
    for r in (again, mixed, fresh):
        for u, v in zip(first, r):
            assert np.array_equal(u, v)
    for u, v in zip(small, small2):
        assert np.array_equal(u, v)
