"""Thin ctypes binding of ``libosann.so`` (C ABI in include/osann.h).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors on the GPU) and
streams.  The functions carry the same names as the C entry points.  There
is no fallback: if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

# OSANN_LIB names another build of the same library (the host sanitizer build of the tests)
LIB_PATH = os.environ.get("OSANN_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libosann.so")

OS_ANN_OK, OS_ANN_EINVAL, OS_ANN_ENOMEM, OS_ANN_EDEVICE, OS_ANN_ENOTSUP, OS_ANN_ENONFINITE = 0, -1, -2, -3, -4, -5
OS_ANN_F32, OS_ANN_F16, OS_ANN_U8 = 0, 1, 2
OS_ANN_MODE_FP32, OS_ANN_MODE_TILED = 0, 1
OS_ANN_FLAG_TIME_KERNELS, OS_ANN_FLAG_GRAPH, OS_ANN_FLAG_BUDGET_CONES = 1, 2, 4
OS_ANN_KERNEL_PROBE, OS_ANN_KERNEL_SCAN, OS_ANN_KERNEL_SCREEN, OS_ANN_KERNEL_FINISH, OS_ANN_KERNEL_GRAPH = 0, 1, 2, 3, 4

_DTYPE_CODE = {torch.float32: OS_ANN_F32, torch.float16: OS_ANN_F16, torch.uint8: OS_ANN_U8}

_lock = threading.Lock()
_lib = None


class OsAnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"osann error {code}: {msg}")
        self.code = code


class os_ann_build_opts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("want_lowp", C.c_int32), ("stream", C.c_void_p)]


class os_ann_search_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("rerank_r", C.c_int32), ("query_dtype", C.c_int32),
                ("flags", C.c_int32), ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_int64), ("walks_capped", C.c_void_p)]


# os_ann_alloc_fn / os_ann_free_fn of os_ann_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

# name -> (restype, argtypes); every symbol include/osann.h declares.
SIGNATURES = {
    "os_ann_build": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32]),
    "os_ann_build_ex": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                     C.POINTER(os_ann_build_opts)]),
    "os_ann_build_rot": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                      C.POINTER(os_ann_build_opts)]),
    "os_ann_build_wht": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                      C.POINTER(os_ann_build_opts)]),
    "os_ann_pca": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.POINTER(os_ann_build_opts),
                             C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_build_proj": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_int32, C.POINTER(os_ann_build_opts)]),
    "os_ann_kmeans": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                C.POINTER(os_ann_build_opts), C.c_void_p]),
    "os_ann_build_ivf": (C.c_void_p, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_int32, C.POINTER(os_ann_build_opts)]),
    "os_ann_set_nprobe": (C.c_int, [C.c_void_p, C.c_int32]),
    "os_ann_search": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "os_ann_search_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                   C.POINTER(os_ann_search_opts), C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_search_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                       C.POINTER(os_ann_search_opts), C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_workspace_bytes": (C.c_int64, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(os_ann_search_opts)]),
    "os_ann_classify": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_export_basis": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "os_ann_export_sparse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_export_rows": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "os_ann_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "os_ann_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "os_ann_free": (None, [C.c_void_p]),
    "os_ann_trim": (C.c_int, []),
    "os_ann_graph_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
    "os_ann_last_tiling": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "os_ann_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, C.c_void_p]),
    "os_ann_last_error": (C.c_int, []),
    "os_ann_last_error_message": (C.c_char_p, []),
    "os_ann_version": (C.c_char_p, []),
}


def lib() -> C.CDLL:
    """Load ``libosann.so``; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_1509_03453_amd.build); "
                                   "there is no fallback path")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _raise(code=None):
    L = lib()
    c = L.os_ann_last_error() if code is None else code
    raise OsAnnError(int(c), (L.os_ann_last_error_message() or b"").decode())


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _check_rows(t: torch.Tensor, what: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous 2-D tensor")
    if t.dtype not in _DTYPE_CODE:
        raise TypeError(f"{what} must be float32, float16 or uint8")
    return _DTYPE_CODE[t.dtype]


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def os_ann_build(db: torch.Tensor, L: int) -> int:
    """Index over FP32 rows ``db[N][D]`` hashed on ``L`` components."""
    if db.dtype != torch.float32:
        raise TypeError("os_ann_build takes float32 rows; use os_ann_build_ex for float16/uint8")
    _check_rows(db, "db")
    h = lib().os_ann_build(_ptr(db), db.shape[0], db.shape[1], int(L))
    if not h:
        _raise()
    return h


def os_ann_build_ex(db: torch.Tensor, L: int, stream=None, want_lowp: bool = False) -> int:
    o = os_ann_build_opts(_check_rows(db, "db"), int(bool(want_lowp)), _stream_ptr(stream))
    h = lib().os_ann_build_ex(_ptr(db), db.shape[0], db.shape[1], int(L), C.byref(o))
    if not h:
        _raise()
    return h


def os_ann_build_rot(db: torch.Tensor, L: int, rot: torch.Tensor, stream=None) -> int:
    """Index with several bases; ``rot`` is a device FP32 tensor [n_rot, D, D]."""
    if rot.dtype != torch.float32 or rot.dim() != 3 or not rot.is_contiguous() or rot.device != db.device:
        raise ValueError("rot must be a contiguous FP32 [n_rot, D, D] tensor on the db's device")
    if rot.shape[1] != db.shape[1] or rot.shape[2] != db.shape[1]:
        raise ValueError("rot must hold D x D matrices")
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    h = lib().os_ann_build_rot(_ptr(db), db.shape[0], db.shape[1], int(L), _ptr(rot), rot.shape[0], C.byref(o))
    if not h:
        _raise()
    return h


def os_ann_build_wht(db: torch.Tensor, L: int, signs: torch.Tensor, stream=None) -> int:
    """Index with several structured bases H diag(s); ``signs`` is a device
    FP32 tensor [n_rot, D] of +-1 (D a power of two)."""
    if signs.dtype != torch.float32 or signs.dim() != 2 or not signs.is_contiguous() or signs.device != db.device:
        raise ValueError("signs must be a contiguous FP32 [n_rot, D] tensor on the db's device")
    if signs.shape[1] != db.shape[1]:
        raise ValueError("signs must hold D entries per basis")
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    h = lib().os_ann_build_wht(_ptr(db), db.shape[0], db.shape[1], int(L), _ptr(signs), signs.shape[0],
                               C.byref(o))
    if not h:
        _raise()
    return h


def os_ann_pca(db: torch.Tensor, k: int, stream=None):
    """Principal axes of the rows of ``db``: ``(mean [D], basis [k, D], var [k])``
    as host numpy arrays (FP32, FP32, float64)."""
    import numpy as np
    D = db.shape[1]
    mean = np.empty(D, dtype=np.float32)
    basis = np.empty((int(k), D), dtype=np.float32)
    var = np.empty(int(k), dtype=np.float64)
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    rc = lib().os_ann_pca(_ptr(db), db.shape[0], D, int(k), C.byref(o), mean.ctypes.data_as(C.c_void_p),
                          basis.ctypes.data_as(C.c_void_p), var.ctypes.data_as(C.c_void_p))
    if rc:
        _raise(rc)
    return mean, basis, var


def os_ann_build_proj(db: torch.Tensor, L: int, basis: torch.Tensor, mean: torch.Tensor | None = None,
                      stream=None) -> int:
    """Index whose cones come from the keys basis (x - mean); ``basis`` is a
    device FP32 tensor [k, D], ``mean`` a device FP32 tensor [D] or None."""
    D = db.shape[1]
    if basis.dtype != torch.float32 or basis.dim() != 2 or not basis.is_contiguous() or basis.device != db.device \
            or basis.shape[1] != D:
        raise ValueError("basis must be a contiguous FP32 [k, D] tensor on the db's device")
    if mean is not None and (mean.dtype != torch.float32 or mean.shape != (D,) or not mean.is_contiguous()
                             or mean.device != db.device):
        raise ValueError("mean must be a contiguous FP32 [D] tensor on the db's device")
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    h = lib().os_ann_build_proj(_ptr(db), db.shape[0], D, int(L), _ptr(mean), _ptr(basis), basis.shape[0],
                                C.byref(o))
    if not h:
        _raise()
    return h


def os_ann_kmeans(db: torch.Tensor, init: torch.Tensor, iters: int, stream=None) -> torch.Tensor:
    """Lloyd k-means from the device FP32 centroids ``init`` [C, D]; returns the new centroids."""
    D = db.shape[1]
    if init.dtype != torch.float32 or init.dim() != 2 or init.shape[1] != D or not init.is_contiguous() \
            or init.device != db.device:
        raise ValueError("init must be a contiguous FP32 [C, D] tensor on the db's device")
    out = torch.empty_like(init)
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    rc = lib().os_ann_kmeans(_ptr(db), db.shape[0], D, init.shape[0], int(iters), _ptr(init), C.byref(o), _ptr(out))
    if rc:
        _raise(rc)
    return out


def os_ann_build_ivf(db: torch.Tensor, L: int, centroids: torch.Tensor, nprobe: int, stream=None) -> int:
    """Clustered index over the device FP32 centroids [C, D]; searches visit ``nprobe`` clusters."""
    D = db.shape[1]
    if centroids.dtype != torch.float32 or centroids.dim() != 2 or centroids.shape[1] != D \
            or not centroids.is_contiguous() or centroids.device != db.device:
        raise ValueError("centroids must be a contiguous FP32 [C, D] tensor on the db's device")
    o = os_ann_build_opts(_check_rows(db, "db"), 0, _stream_ptr(stream))
    h = lib().os_ann_build_ivf(_ptr(db), db.shape[0], D, int(L), _ptr(centroids), centroids.shape[0], int(nprobe),
                               C.byref(o))
    if not h:
        _raise()
    return h


def os_ann_set_nprobe(index: int, nprobe: int) -> None:
    rc = lib().os_ann_set_nprobe(index, int(nprobe))
    if rc:
        _raise(rc)


def _search_opts(queries, mode, stream, workspace, rerank_r=8, flags=0, walks_capped=None):
    qt = _check_rows(queries, "queries") if queries is not None else OS_ANN_F32
    ws = 0 if workspace is None else workspace.numel() * workspace.element_size()
    if walks_capped is not None and (walks_capped.dtype != torch.int64 or not walks_capped.is_cuda):
        raise ValueError("walks_capped must be a GPU int64 tensor")
    return os_ann_search_opts(int(mode), int(rerank_r), qt, int(flags), _stream_ptr(stream),
                              _ptr(workspace), int(ws), _ptr(walks_capped))


def os_ann_search(index: int, queries: torch.Tensor, max_candidates: int,
                  out_idx: torch.Tensor | None = None, out_dist: torch.Tensor | None = None):
    """NN of FP32 queries on the current stream: ``(idx int64[Q], dist float32[Q])``."""
    if queries.dtype != torch.float32:
        raise TypeError("os_ann_search takes float32 queries; use os_ann_search_ex")
    _check_rows(queries, "queries")
    Q = queries.shape[0]
    out_idx = torch.empty(Q, dtype=torch.int64, device=queries.device) if out_idx is None else out_idx
    out_dist = torch.empty(Q, dtype=torch.float32, device=queries.device) if out_dist is None else out_dist
    if torch.cuda.current_stream().cuda_stream != 0:
        # the plain call runs on the null stream; keep torch's ordering
        torch.cuda.current_stream().synchronize()
    rc = lib().os_ann_search(index, _ptr(queries), Q, int(max_candidates), _ptr(out_idx), _ptr(out_dist))
    if rc:
        _raise(rc)
    return out_idx, out_dist


def os_ann_search_ex(index: int, queries: torch.Tensor, max_candidates: int, mode: int = OS_ANN_MODE_FP32,
                     stream=None, workspace: torch.Tensor | None = None, rerank_r: int = 8,
                     out_idx=None, out_dist=None, out_ncand=None, want_ncand: bool = True,
                     flags: int = 0, cones: bool = False, walks_capped: torch.Tensor | None = None):
    """As os_ann_search with options; returns ``(idx, dist, ncand or None)``.
    ``cones``: max_candidates is the number C of cones each walk takes
    (OS_ANN_FLAG_BUDGET_CONES).  ``walks_capped`` (one GPU int64, sparse
    tables): receives the number of walks the position cap stopped."""
    if cones:
        flags |= OS_ANN_FLAG_BUDGET_CONES
    o = _search_opts(queries, mode, stream, workspace, rerank_r, flags, walks_capped)
    Q = queries.shape[0]
    dev = queries.device
    out_idx = torch.empty(Q, dtype=torch.int64, device=dev) if out_idx is None else out_idx
    out_dist = torch.empty(Q, dtype=torch.float32, device=dev) if out_dist is None else out_dist
    if out_ncand is None and want_ncand:
        out_ncand = torch.empty(Q, dtype=torch.int64, device=dev)
    rc = lib().os_ann_search_ex(index, _ptr(queries), Q, int(max_candidates), C.byref(o),
                                _ptr(out_idx), _ptr(out_dist), _ptr(out_ncand))
    if rc:
        _raise(rc)
    return out_idx, out_dist, out_ncand


def os_ann_search_static(index: int, queries: torch.Tensor, max_candidates: int, out_idx: torch.Tensor,
                         out_dist: torch.Tensor, out_ncand: torch.Tensor | None = None, stream=None,
                         cones: bool = False) -> None:
    """FP32 search into caller-owned outputs with the library's fixed device
    scratch (no allocation by the library)."""
    o = _search_opts(queries, OS_ANN_MODE_FP32, stream, None, 8, OS_ANN_FLAG_BUDGET_CONES if cones else 0)
    Q = queries.shape[0]
    for t, dt, what in ((out_idx, torch.int64, "out_idx"), (out_dist, torch.float32, "out_dist"),
                        (out_ncand, torch.int64, "out_ncand")):
        if t is not None and (t.dtype != dt or t.numel() < Q or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{what} must be a contiguous GPU {dt} tensor of at least {Q} elements")
    rc = lib().os_ann_search_static(index, _ptr(queries), Q, int(max_candidates), C.byref(o),
                                    _ptr(out_idx), _ptr(out_dist), _ptr(out_ncand))
    if rc:
        _raise(rc)


def os_ann_workspace_bytes(index: int, Q: int, max_candidates: int, mode: int = OS_ANN_MODE_FP32,
                           rerank_r: int = 8, cones: bool = False) -> int:
    o = os_ann_search_opts(int(mode), int(rerank_r), OS_ANN_F32, OS_ANN_FLAG_BUDGET_CONES if cones else 0,
                           None, None, 0)
    n = lib().os_ann_workspace_bytes(index, int(Q), int(max_candidates), C.byref(o))
    if n < 0:
        _raise(n)
    return int(n)


def os_ann_classify(index: int, queries: torch.Tensor, max_candidates: int, stream=None):
    """Own cone (int64 view of uint32), packed top-L pairs and candidate counts."""
    qt = _check_rows(queries, "queries")
    Q = queries.shape[0]
    dev = queries.device
    cone = torch.empty(Q, dtype=torch.int32, device=dev)
    top = torch.empty(Q, dtype=torch.int64, device=dev)
    ncand = torch.empty(Q, dtype=torch.int64, device=dev)
    rc = lib().os_ann_classify(index, _ptr(queries), qt, Q, int(max_candidates), _ptr(cone), _ptr(top),
                               _ptr(ncand), _stream_ptr(stream))
    if rc:
        _raise(rc)
    return cone, top, ncand


def os_ann_kernel_time(index: int, kernel: int) -> tuple[int, float]:
    """(launches, total milliseconds) of timed launches of one kernel; clears them."""
    n, ms = C.c_int64(), C.c_double()
    rc = lib().os_ann_kernel_time(index, int(kernel), C.byref(n), C.byref(ms))
    if rc:
        _raise(rc)
    return int(n.value), float(ms.value)


def os_ann_info(index: int) -> dict:
    N, D, L = C.c_int64(), C.c_int32(), C.c_int32()
    nc, ne, nb = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().os_ann_info(index, C.byref(N), C.byref(D), C.byref(L), C.byref(nc), C.byref(ne), C.byref(nb))
    if rc:
        _raise(rc)
    return {"N": N.value, "D": D.value, "L": L.value, "n_cones": nc.value, "n_nonempty": ne.value,
            "device_bytes": nb.value}


def os_ann_graph_stats(index: int) -> dict:
    """Graphs captured, graph replays and graphs kept by an index."""
    cap, rep, kept = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().os_ann_graph_stats(index, C.byref(cap), C.byref(rep), C.byref(kept))
    if rc:
        _raise(rc)
    return {"captured": cap.value, "replayed": rep.value, "cached": kept.value}


def os_ann_last_tiling(index: int) -> dict:
    """Kernel (0 query-tile, 1 cone-major), query order, groups and splits of the last tiled search."""
    k, o, g, sp = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    rc = lib().os_ann_last_tiling(index, C.byref(k), C.byref(o), C.byref(g), C.byref(sp))
    if rc:
        _raise(rc)
    return {"kernel": k.value, "order": o.value, "groups": g.value, "splits": sp.value}


def os_ann_export(index: int, stream=None) -> dict:
    """Row cones (int32 view of uint32), packed top-L, offsets and perm."""
    info = os_ann_info(index)
    N, nc = info["N"], info["n_cones"]
    if nc > (1 << 24):  # only sparse tables have more cones than dense offsets address
        raise OsAnnError(OS_ANN_ENOTSUP, "sparse table: use os_ann_export_sparse")
    dev = torch.device("cuda", torch.cuda.current_device())
    cone = torch.empty(N, dtype=torch.int32, device=dev)
    top = torch.empty(N, dtype=torch.int64, device=dev)
    off = torch.empty(nc + 1, dtype=torch.int64, device=dev)
    perm = torch.empty(N, dtype=torch.int64, device=dev)
    rc = lib().os_ann_export(index, _ptr(cone), _ptr(top), _ptr(off), _ptr(perm), _stream_ptr(stream))
    if rc:
        _raise(rc)
    return {"cone": cone, "top": top, "offsets": off, "perm": perm}


def os_ann_export_basis(index: int, r: int, stream=None) -> dict:
    """As os_ann_export, for basis ``r`` of a several-bases index."""
    info = os_ann_info(index)
    N, nc = info["N"], info["n_cones"]
    dev = torch.device("cuda", torch.cuda.current_device())
    cone = torch.empty(N, dtype=torch.int32, device=dev)
    top = torch.empty(N, dtype=torch.int64, device=dev)
    off = torch.empty(nc + 1, dtype=torch.int64, device=dev)
    perm = torch.empty(N, dtype=torch.int64, device=dev)
    rc = lib().os_ann_export_basis(index, int(r), _ptr(cone), _ptr(top), _ptr(off), _ptr(perm),
                                   _stream_ptr(stream))
    if rc:
        _raise(rc)
    return {"cone": cone, "top": top, "offsets": off, "perm": perm}


def os_ann_export_sparse(index: int, stream=None) -> dict:
    """Sparse table: distinct cone ids (int64 view of uint64), their row
    offsets, the permutation and the packed top-L pairs of the rows."""
    info = os_ann_info(index)
    N, ne = info["N"], info["n_nonempty"]
    dev = torch.device("cuda", torch.cuda.current_device())
    ids = torch.empty(ne, dtype=torch.int64, device=dev)
    off = torch.empty(ne + 1, dtype=torch.int64, device=dev)
    perm = torch.empty(N, dtype=torch.int64, device=dev)
    top = torch.empty(N, dtype=torch.int64, device=dev)
    rc = lib().os_ann_export_sparse(index, _ptr(ids), _ptr(off), _ptr(perm), _stream_ptr(stream))
    if rc:
        _raise(rc)
    rc = lib().os_ann_export(index, None, _ptr(top), None, None, _stream_ptr(stream))
    if rc:
        _raise(rc)
    return {"cone_ids": ids, "offsets": off, "perm": perm, "top": top}


def os_ann_export_rows(index: int, stream=None) -> torch.Tensor:
    info = os_ann_info(index)
    rows = torch.empty(info["N"], info["D"], dtype=torch.float32,
                       device=torch.device("cuda", torch.cuda.current_device()))
    rc = lib().os_ann_export_rows(index, _ptr(rows), _stream_ptr(stream))
    if rc:
        _raise(rc)
    return rows


def os_ann_free(index: int) -> None:
    if index:
        lib().os_ann_free(index)


def os_ann_trim() -> None:
    """Hand the library's idle device blocks back to the HIP runtime."""
    lib().os_ann_trim()


_hooks = None  # the ctypes callbacks in use (kept alive while the library holds them)


def os_ann_set_allocator(alloc=None, free=None) -> None:
    """Route the library's device allocations through ``alloc(nbytes,
    stream_ptr) -> device pointer (int, 0 when out of memory)`` and
    ``free(ptr, stream_ptr)``; ``None, None`` restores the library's own."""
    global _hooks
    if (alloc is None) != (free is None):
        raise ValueError("give both functions or neither")
    if alloc is None:
        rc = lib().os_ann_set_allocator(C.cast(None, ALLOC_FN), C.cast(None, FREE_FN), None)
        if rc:
            _raise(rc)
        _hooks = None
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:  # an exception must not cross the C boundary: report no memory
            return None

    def _free(ptr, stream, ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:
            pass

    hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
    rc = lib().os_ann_set_allocator(hooks[0], hooks[1], None)
    if rc:
        _raise(rc)
    _hooks = hooks


def use_torch_allocator() -> None:
    """Let PyTorch's caching allocator own the library's device memory."""
    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    os_ann_set_allocator(alloc, free)


def os_ann_last_error() -> int:
    return int(lib().os_ann_last_error())


def os_ann_last_error_message() -> str:
    return (lib().os_ann_last_error_message() or b"").decode()


def os_ann_version() -> str:
    return lib().os_ann_version().decode()


class Index:
    """Owning wrapper of an index handle (frees it when collected)."""

    def __init__(self, db: torch.Tensor, L: int, stream=None, want_lowp: bool = False):
        self.handle = os_ann_build_ex(db, L, stream=stream, want_lowp=want_lowp)
        self.info = os_ann_info(self.handle)

    def search(self, queries, max_candidates, mode=OS_ANN_MODE_FP32, stream=None, workspace=None,
               rerank_r=8):
        return os_ann_search_ex(self.handle, queries, max_candidates, mode=mode, stream=stream,
                                workspace=workspace, rerank_r=rerank_r)

    def workspace_bytes(self, Q, max_candidates, mode=OS_ANN_MODE_FP32, rerank_r=8):
        return os_ann_workspace_bytes(self.handle, Q, max_candidates, mode, rerank_r)

    def classify(self, queries, max_candidates, stream=None):
        return os_ann_classify(self.handle, queries, max_candidates, stream=stream)

    def export(self, stream=None):
        return os_ann_export(self.handle, stream=stream)

    def close(self):
        if getattr(self, "handle", None):
            os_ann_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
