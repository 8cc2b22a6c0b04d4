"""Helpers of the GPU parity tests: move arrays, call the C ABI through the
binding, decode its packed outputs.  Nothing here computes the method."""
import sys

import numpy as np
import torch

from paper_1509_03453_amd import binding as B


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def unpack_top(packed: np.ndarray, L: int):
    p = packed.astype(np.uint64)
    idx = np.stack([((p >> np.uint64(9 * j)) & np.uint64(0xFF)).astype(np.int64) for j in range(L)], 1)
    sg = np.stack([((p >> np.uint64(9 * j + 8)) & np.uint64(1)).astype(np.uint8) for j in range(L)], 1)
    return idx, sg


def gpu_index(X: np.ndarray, L: int):
    """Build through the C ABI; returns (handle, exported arrays as numpy)."""
    h = B.os_ann_build_ex(dev(X), L)
    ex = B.os_ann_export(h)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in ex.items()}
    out["cone"] = out["cone"].view(np.uint32).astype(np.int64)
    out["top_idx"], out["top_sign"] = unpack_top(out["top"].view(np.uint64), L)
    return h, out


def gpu_search(h, Y: np.ndarray, budget: int, mode=B.OS_ANN_MODE_FP32):
    i, d, n = B.os_ann_search_ex(h, dev(Y), budget, mode=mode)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy(), n.cpu().numpy()
