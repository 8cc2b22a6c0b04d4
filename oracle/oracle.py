"""ctypes front-end of the plain CPU oracle (``osann_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product library.  It shares
no code with the GPU path; it only receives the same numpy input arrays.

Notation (paper): ``K`` vector length, ``G`` number of largest components
hashed, ``N_C = C(K,G) 2^G`` cones.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "osann_oracle.c")
_lock = threading.Lock()
_lib = None

DTYPES = {np.dtype(np.float32): 0, np.dtype(np.float16): 1, np.dtype(np.uint8): 2}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def _host_tag() -> str:
    # the library is compiled for the CPU it runs on (-march=native), so it
    # is kept per CPU model and instruction-set flags
    flags = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    flags = line
                    break
    except OSError:
        pass
    return hashlib.sha1((cpu_model() + flags).encode()).hexdigest()[:12]


_LIB = os.path.join(_HERE, f"libosann_oracle.{_host_tag()}.so")
# A separately built copy (the sanitizer build of the tests) may stand in.
_LIB_OVERRIDE = os.environ.get("OSANN_ORACLE_LIB")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc for this host's CPU: -O3 -march=native,
    no fused or re-associated FP arithmetic (-ffp-contract=off, no fast math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-std=c11", "-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (every finding aborts) into ``out``, for the host sanitizer test."""
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fPIC", "-shared",
           "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                L = C.CDLL(_LIB_OVERRIDE)
            else:
                build()
                L = C.CDLL(_LIB)
            p = C.c_void_p
            i64, i32 = C.c_int64, C.c_int
            L.orc_binom.restype = i64
            L.orc_binom.argtypes = [i32, i32]
            L.orc_num_cones.restype = i64
            L.orc_num_cones.argtypes = [i32, i32]
            L.orc_rank_order.restype = None
            L.orc_rank_order.argtypes = [p, i32, p]
            L.orc_hash.restype = i32
            L.orc_hash.argtypes = [p, i32, i64, i32, i32, p, p, p]
            L.orc_bucket.restype = i32
            L.orc_bucket.argtypes = [p, i64, i64, p, p]
            L.orc_walk.restype = i64
            L.orc_walk.argtypes = [p, i32, i32, p, i64]
            L.orc_probe.restype = i64
            L.orc_probe.argtypes = [p, i32, i32, p, i64, p, i64, p]
            L.orc_probe_cones.restype = i64
            L.orc_probe_cones.argtypes = [p, i32, i32, p, i64, p, i64, p]
            L.orc_search.restype = i32
            L.orc_search.argtypes = [p, i32, i64, i32, i32, p, p, p, i32, i64, i64, p, p, p, p, i32]
            L.orc_exhaustive.restype = i32
            L.orc_exhaustive.argtypes = [p, i32, i64, i32, p, i32, i64, p, p, p, p, i32]
            L.orc_pair_d64.restype = i32
            L.orc_pair_d64.argtypes = [p, i32, i32, p, i32, p, i64, p]
            L.orc_pair_d32.restype = i32
            L.orc_pair_d32.argtypes = [p, i32, i32, p, i32, p, i64, p]
            L.orc_search_tiled.restype = i32
            L.orc_search_tiled.argtypes = [p, i32, i64, i32, i32, p, p, p, i32, i64, i64, i32, i32,
                                           p, p, p, p, p, p, i32, i32, p, i32]
            L.orc_pair_dtilde.restype = i32
            L.orc_pair_dtilde.argtypes = [p, i32, i32, p, i32, p, i64, i32, p]
            L.orc_round_short.restype = i32
            L.orc_round_short.argtypes = [p, i64, i32, p]
            L.orc_rotate.restype = i32
            L.orc_rotate.argtypes = [p, i32, i64, i32, p, p]
            L.orc_search_rot.restype = i32
            L.orc_search_rot.argtypes = [p, i32, i64, i32, i32, i32, p, p, p, p, i32, i64, i64,
                                         p, p, p, p, i32, i32, i32]
            L.orc_wht.restype = i32
            L.orc_wht.argtypes = [p, i32, i64, i32, p, p]
            L.orc_bucket_sparse.restype = i64
            L.orc_bucket_sparse.argtypes = [p, i64, p, p, p]
            L.orc_walk_prefix.restype = i64
            L.orc_walk_prefix.argtypes = [p, i32, i32, p, i64]
            L.orc_search_sparse.restype = i32
            L.orc_search_sparse.argtypes = [p, i32, i64, i32, i32, p, i64, p, p, p, i32, i64, i64, i32,
                                            p, p, p, p, i32]
            L.orc_search_keyed.restype = i32
            L.orc_search_keyed.argtypes = [p, i32, i64, i32, i32, i32, p, p, p, i32, p, i64, i64,
                                           p, p, p, p, i32, i32]
            L.orc_project.restype = i32
            L.orc_project.argtypes = [p, i32, i64, i32, p, p, i32, p]
            L.orc_assign.restype = i32
            L.orc_assign.argtypes = [p, i32, i64, i32, p, i32, p]
            L.orc_kmeans_update.restype = i32
            L.orc_kmeans_update.argtypes = [p, i32, i64, i32, p, i32, p, p]
            L.orc_search_ivf.restype = i32
            L.orc_search_ivf.argtypes = [p, i32, i64, i32, i32, p, i32, p, p, p, i32, i64, i64, i32,
                                         p, p, p, p, i32, i32]
            _lib = L
    return _lib


def _arr(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return a, a.ctypes.data_as(C.c_void_p)


def _rows(a):
    a = np.ascontiguousarray(a)
    if a.dtype not in DTYPES:
        raise TypeError(f"oracle rows must be float32, float16 or uint8, not {a.dtype}")
    if a.ndim != 2:
        raise ValueError("oracle rows must be 2-D")
    return a, a.ctypes.data_as(C.c_void_p), DTYPES[a.dtype]


def binom(n: int, k: int) -> int:
    return int(lib().orc_binom(n, k))


def num_cones(K: int, G: int) -> int:
    """N_C = C(K,G) 2^G (Section 2, Table I)."""
    return int(lib().orc_num_cones(K, G))


def rank_order(v) -> np.ndarray:
    """Indices of ``v`` by decreasing magnitude, ties to the lower index."""
    v, pv = _arr(v, np.float32)
    out = np.empty(v.shape[0], dtype=np.int32)
    lib().orc_rank_order(pv, v.shape[0], out.ctypes.data_as(C.c_void_p))
    return out


def hash_rows(X, G: int):
    """Per row: top-G indices (decreasing magnitude), their sign bits, cone id."""
    X, px, dt = _rows(X)
    N, K = X.shape
    top = np.empty((N, G), dtype=np.int32)
    sg = np.empty((N, G), dtype=np.uint8)
    cone = np.empty(N, dtype=np.int64)
    rc = lib().orc_hash(px, dt, N, K, G, top.ctypes.data_as(C.c_void_p),
                        sg.ctypes.data_as(C.c_void_p), cone.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_hash failed ({rc})")
    return top, sg, cone


def bucket(cone, n_cones: int):
    """Stable counting sort by cone: ``(offsets[N_C+1], perm[N])``."""
    cone, pc = _arr(cone, np.int64)
    off = np.empty(n_cones + 1, dtype=np.int64)
    perm = np.empty(cone.shape[0], dtype=np.int64)
    rc = lib().orc_bucket(pc, cone.shape[0], n_cones, off.ctypes.data_as(C.c_void_p),
                          perm.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_bucket failed ({rc})")
    return off, perm


def build_index(X, G: int):
    """Hash + bucket: dict with top, sign, cone, offsets, perm, n_cones."""
    K = X.shape[1]
    nc = num_cones(K, G)
    top, sg, cone = hash_rows(X, G)
    off, perm = bucket(cone, nc)
    return {"top": top, "sign": sg, "cone": cone, "offsets": off, "perm": perm,
            "n_cones": nc, "K": K, "G": G}


def walk(y, G: int) -> np.ndarray:
    """All N_C cones of one query, in probe order (empty ones included)."""
    y, py = _arr(y, np.float32)
    K = y.shape[0]
    nc = num_cones(K, G)
    out = np.empty(nc, dtype=np.int64)
    n = lib().orc_walk(py, K, G, out.ctypes.data_as(C.c_void_p), nc)
    assert n == nc, (n, nc)
    return out


def probe(y, G: int, offsets, B: int):
    """Non-empty cones probed within budget ``B`` and the candidate count."""
    y, py = _arr(y, np.float32)
    off, po = _arr(offsets, np.int64)
    K = y.shape[0]
    nc = off.shape[0] - 1
    out = np.empty(nc, dtype=np.int64)
    nca = np.zeros(1, dtype=np.int64)
    n = lib().orc_probe(py, K, G, po, int(B), out.ctypes.data_as(C.c_void_p), nc,
                        nca.ctypes.data_as(C.c_void_p))
    return out[:n].copy(), int(nca[0])


def probe_cones(y, G: int, offsets, n_take: int):
    """Fixed-C mode (reading R13): the non-empty cones among the first
    ``n_take`` (the paper's C) cones of the walk, and their candidate count."""
    y, py = _arr(y, np.float32)
    off, po = _arr(offsets, np.int64)
    K = y.shape[0]
    nc = off.shape[0] - 1
    out = np.empty(nc, dtype=np.int64)
    nca = np.zeros(1, dtype=np.int64)
    n = lib().orc_probe_cones(py, K, G, po, int(n_take), out.ctypes.data_as(C.c_void_p), nc,
                              nca.ctypes.data_as(C.c_void_p))
    return out[:n].copy(), int(nca[0])


def search(X, index, Y, B: int, nthreads: int = 0, cones: bool = False):
    """Algorithm 1 with one basis: ``(idx, d32, d64, ncand)`` per query.
    With ``cones`` the budget ``B`` counts cones (reading R13)."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    off, po = _arr(index["offsets"], np.int64)
    perm, pp = _arr(index["perm"], np.int64)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    rc = lib().orc_search_keyed(px, xdt, N, K, K, index["G"], po, pp, py, ydt, None, Q, int(B),
                                idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                                d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p),
                                int(nthreads), int(bool(cones)))
    if rc != 0:
        raise RuntimeError(f"orc_search failed ({rc})")
    return idx, d32, d64, nca


def exhaustive(X, Y, nthreads: int = 0):
    """Exact NN (eq. (1)): ``(idx32, d32, idx64, d64)`` per query."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    i32 = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    i64 = np.empty(Q, dtype=np.int64)
    d64 = np.empty(Q, dtype=np.float64)
    lib().orc_exhaustive(px, xdt, N, K, py, ydt, Q, i32.ctypes.data_as(C.c_void_p),
                         d32.ctypes.data_as(C.c_void_p), i64.ctypes.data_as(C.c_void_p),
                         d64.ctypes.data_as(C.c_void_p), int(nthreads))
    return i32, d32, i64, d64


def pair_d64(X, Y, rows) -> np.ndarray:
    """Double squared distance between query q and row ``rows[q]``."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    r, pr = _arr(rows, np.int64)
    out = np.empty(Y.shape[0], dtype=np.float64)
    lib().orc_pair_d64(px, xdt, X.shape[1], py, ydt, pr, Y.shape[0], out.ctypes.data_as(C.c_void_p))
    return out


def pair_d32(X, Y, rows) -> np.ndarray:
    """FP32 squared distance (term by term, i ascending) of (q, rows[q])."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    r, pr = _arr(rows, np.int64)
    out = np.empty(Y.shape[0], dtype=np.float32)
    lib().orc_pair_d32(px, xdt, X.shape[1], py, ydt, pr, Y.shape[0], out.ctypes.data_as(C.c_void_p))
    return out


def search_tiled(X, index, Y, B: int, R: int = 8, use_f16: bool | None = None, nthreads: int = 0,
                 cones: bool = False):
    """Screened search (reading R7): ``(idx, d32, d64, ncand, dt_R, top)``.
    With ``cones`` the budget ``B`` counts cones (reading R13).  On a keyed
    table (``index`` from build_index_proj) the walk runs on the queries'
    keys and the screen on the full queries (reading R11).

    ``use_f16`` defaults to True for float16 rows (the rows are kept as
    stored) and False otherwise (bfloat16 rounding)."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    if use_f16 is None:
        use_f16 = X.dtype == np.float16
    N, K = X.shape
    Q = Y.shape[0]
    if index.get("P") is not None:  # keyed table: walk on the keys
        Yk = np.ascontiguousarray(project(Y, index["mu"], index["P"]), dtype=np.float32)
        pk, kk = Yk.ctypes.data_as(C.c_void_p), Yk.shape[1]
    else:
        Yk, pk, kk = None, None, K
    off, po = _arr(index["offsets"], np.int64)
    perm, pp = _arr(index["perm"], np.int64)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    dtr = np.empty(Q, dtype=np.float64)
    top = np.empty((Q, R), dtype=np.int64)
    rc = lib().orc_search_tiled(px, xdt, N, K, index["G"], po, pp, py, ydt, Q, int(B), int(R), int(use_f16),
                                idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                                d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p),
                                dtr.ctypes.data_as(C.c_void_p), top.ctypes.data_as(C.c_void_p), int(nthreads),
                                int(bool(cones)), pk, kk)
    if rc != 0:
        raise RuntimeError(f"orc_search_tiled failed ({rc})")
    return idx, d32, d64, nca, dtr, top


def pair_dtilde(X, Y, rows, use_f16: bool = False) -> np.ndarray:
    """d~ = ||x^||^2 - 2 q^.x^ of (q, rows[q]) in double on rounded values."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    r, pr = _arr(rows, np.int64)
    out = np.empty(Y.shape[0], dtype=np.float64)
    lib().orc_pair_dtilde(px, xdt, X.shape[1], py, ydt, pr, Y.shape[0], int(use_f16),
                          out.ctypes.data_as(C.c_void_p))
    return out


def round_short(x, use_f16: bool = False) -> np.ndarray:
    """Values rounded to bfloat16 (or binary16), as doubles."""
    x, px = _arr(np.ravel(x), np.float32)
    out = np.empty(x.shape[0], dtype=np.float64)
    lib().orc_round_short(px, x.shape[0], int(use_f16), out.ctypes.data_as(C.c_void_p))
    return out


def rotate(X, M):
    """Coordinates of the rows of ``X`` in the basis ``M`` (K x K), FP32 (reading R9)."""
    X, px, dt = _rows(X)
    N, K = X.shape
    M, pm = _arr(M, np.float32)
    out = np.empty((N, K), dtype=np.float32)
    rc = lib().orc_rotate(px, dt, N, K, pm, out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_rotate failed ({rc})")
    return out


def wht(X, signs):
    """Coordinates in the structured basis H diag(signs) (fast Walsh-Hadamard
    transform in FP32, unnormalised; reading R14)."""
    X, px, dt = _rows(X)
    N, K = X.shape
    sg, ps = _arr(signs, np.float32)
    if sg.shape != (K,):
        raise ValueError("signs must have one entry per component")
    out = np.empty((N, K), dtype=np.float32)
    rc = lib().orc_wht(px, dt, N, K, ps, out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_wht failed ({rc})")
    return out


def build_index_wht(X, G: int, signs):
    """Several structured bases (reading R14): basis r is H diag(signs[r])."""
    signs = np.ascontiguousarray(signs, dtype=np.float32)
    tabs = [build_index(wht(X, signs[r]), G) for r in range(signs.shape[0])]
    return {"tables": tabs, "rots": signs, "wht": True, "G": G, "K": X.shape[1], "n_cones": tabs[0]["n_cones"]}


def build_index_rot(X, G: int, rots):
    """One table per basis (Section 3.A): the rows' coordinates in basis r
    are hashed and bucketed; every table refers to the original rows."""
    rots = np.ascontiguousarray(rots, dtype=np.float32)
    tabs = [build_index(rotate(X, rots[r]), G) for r in range(rots.shape[0])]
    return {"tables": tabs, "rots": rots, "G": G, "K": X.shape[1], "n_cones": tabs[0]["n_cones"]}


def search_rot(X, index, Y, B: int, nthreads: int = 0, cones: bool = False):
    """Algorithm 1 with several bases: ``(idx, d32, d64, ncand)`` per query.
    With ``cones`` the search visits levels 0..B-1 of every basis (reading R13)."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    R = len(index["tables"])
    off, po = _arr(np.concatenate([t["offsets"] for t in index["tables"]]), np.int64)
    perm, pp = _arr(np.concatenate([t["perm"] for t in index["tables"]]), np.int64)
    rots, pr = _arr(index["rots"], np.float32)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    rc = lib().orc_search_rot(px, xdt, N, K, index["G"], R, pr, po, pp, py, ydt, Q, int(B),
                              idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                              d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p),
                              int(nthreads), int(bool(cones)), int(bool(index.get("wht", False))))
    if rc != 0:
        raise RuntimeError(f"orc_search_rot failed ({rc})")
    return idx, d32, d64, nca


# ---------------------------------------------------------------------------
# PCA front-end (Section 4.B; reading R11)
# ---------------------------------------------------------------------------

def pca_basis(X, k: int):
    """Principal axes of the rows: the float64 mean and covariance (sum of the
    centred outer products divided by N), their eigen-decomposition
    (``numpy.linalg.eigh``), the k axes of largest variance in decreasing
    order, each signed so that its largest-magnitude component (lowest index
    on ties) is positive.  Returns ``(mu, P, lam)``: FP32 mean (K), FP32 axes
    (k x K, one per row) and their float64 variances."""
    Xd = np.asarray(X).astype(np.float64)
    N, K = Xd.shape
    if not 1 <= k <= K:
        raise ValueError("k must be in [1, K]")
    mu = Xd.mean(axis=0)
    Xc = Xd - mu
    cov = Xc.T @ Xc / N
    lam, V = np.linalg.eigh(cov)
    pick = np.argsort(-lam, kind="stable")[:k]
    P = V[:, pick].T.copy()
    for i in range(k):
        j = int(np.argmax(np.abs(P[i])))
        if P[i, j] < 0:
            P[i] = -P[i]
    return mu.astype(np.float32), P.astype(np.float32), lam[pick]


def project(X, mu, P):
    """Keys P (x - mu) of the rows of ``X`` in FP32 term by term (reading R11);
    ``mu`` may be None (no centring)."""
    X, px, dt = _rows(X)
    N, K = X.shape
    P, pp = _arr(P, np.float32)
    k = P.shape[0]
    if P.shape[1] != K:
        raise ValueError("P must be k x K")
    if mu is None:
        pm = None
    else:
        mu, pm = _arr(mu, np.float32)
    out = np.empty((N, k), dtype=np.float32)
    rc = lib().orc_project(px, dt, N, K, pm, pp, k, out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_project failed ({rc})")
    return out


def build_index_proj(X, G: int, mu, P):
    """One table built from the rows' keys P (x - mu); distances stay on the rows."""
    idx = build_index(project(X, mu, P), G)
    idx["mu"] = None if mu is None else np.ascontiguousarray(mu, dtype=np.float32)
    idx["P"] = np.ascontiguousarray(P, dtype=np.float32)
    return idx


def search_proj(X, index, Y, B: int, nthreads: int = 0, cones: bool = False):
    """Algorithm 1 on a keyed table: each query walks the cones of its own key,
    candidates are compared on all components.  ``(idx, d32, d64, ncand)``."""
    Yk = project(Y, index["mu"], index["P"])
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    Kk = Yk.shape[1]
    off, po = _arr(index["offsets"], np.int64)
    perm, pp = _arr(index["perm"], np.int64)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    rc = lib().orc_search_keyed(px, xdt, N, K, Kk, index["G"], po, pp, py, ydt,
                                Yk.ctypes.data_as(C.c_void_p), Q, int(B),
                                idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                                d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p),
                                int(nthreads), int(bool(cones)))
    if rc != 0:
        raise RuntimeError(f"orc_search_keyed failed ({rc})")
    return idx, d32, d64, nca


# ---------------------------------------------------------------------------
# Coarse clusters (ROSANNA+, Section 4.B; reading R12)
# ---------------------------------------------------------------------------

def assign(X, cent):
    """Nearest centroid of each row (FP32 term-by-term distance, lower id on ties)."""
    X, px, dt = _rows(X)
    N, K = X.shape
    cent, pc = _arr(cent, np.float32)
    out = np.empty(N, dtype=np.int32)
    rc = lib().orc_assign(px, dt, N, K, pc, cent.shape[0], out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError(f"orc_assign failed ({rc})")
    return out


def kmeans(X, init, iters: int):
    """Lloyd k-means from ``init`` (C x K FP32) for ``iters`` iterations;
    returns the FP32 centroids."""
    X, px, dt = _rows(X)
    N, K = X.shape
    cent = np.ascontiguousarray(init, dtype=np.float32).copy()
    for _ in range(int(iters)):
        a = assign(X, cent)
        new = np.empty_like(cent)
        rc = lib().orc_kmeans_update(px, dt, N, K, a.ctypes.data_as(C.c_void_p), cent.shape[0],
                                     cent.ctypes.data_as(C.c_void_p), new.ctypes.data_as(C.c_void_p))
        if rc != 0:
            raise ValueError(f"orc_kmeans_update failed ({rc})")
        cent = new
    return cent


def build_index_ivf(X, G: int, cent):
    """Rows bucketed by (cluster, cone of the residual x - c): bucket id
    cluster * N_C + cone, offsets over C * N_C buckets."""
    cent = np.ascontiguousarray(cent, dtype=np.float32)
    a = assign(X, cent)
    R = np.asarray(X).astype(np.float32) - cent[a]
    top, sg, cone = hash_rows(R, G)
    nc = num_cones(X.shape[1], G)
    comp = a.astype(np.int64) * nc + cone
    off, perm = bucket(comp, nc * cent.shape[0])
    return {"top": top, "sign": sg, "cone": comp, "assign": a, "offsets": off, "perm": perm,
            "n_cones": nc, "K": X.shape[1], "G": G, "cent": cent}


def search_ivf(X, index, Y, B: int, nprobe: int, nthreads: int = 0, cones: bool = False):
    """Search in the nprobe nearest clusters: ``(idx, d32, d64, ncand)``.
    With ``cones`` each searched cluster takes the first B cones of its walk
    (reading R13)."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    cent, pc = _arr(index["cent"], np.float32)
    off, po = _arr(index["offsets"], np.int64)
    perm, pp = _arr(index["perm"], np.int64)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    rc = lib().orc_search_ivf(px, xdt, N, K, index["G"], pc, cent.shape[0], po, pp, py, ydt, Q, int(B),
                              int(nprobe), idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                              d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p), int(nthreads),
                              int(bool(cones)))
    if rc != 0:
        raise RuntimeError(f"orc_search_ivf failed ({rc})")
    return idx, d32, d64, nca


# ---------------------------------------------------------------------------
# Sparse table (Section 4, second-level hash; reading R15)
# ---------------------------------------------------------------------------

def walk_prefix(y, G: int, n: int) -> np.ndarray:
    """The first ``n`` cones of the query's walk (Section 3.B), empty or not."""
    y, py = _arr(y, np.float32)
    out = np.empty(int(n), dtype=np.int64)
    m = lib().orc_walk_prefix(py, y.shape[0], G, out.ctypes.data_as(C.c_void_p), int(n))
    return out[:m].copy()


def build_index_sparse(X, G: int):
    """Rows hashed as for one basis, then kept as a sparse table: the distinct
    non-empty cones in ascending order (``keys``) and their rows' offsets."""
    top, sg, cone = hash_rows(X, G)
    N = cone.shape[0]
    keys = np.empty(N, dtype=np.int64)
    off = np.empty(N + 1, dtype=np.int64)
    perm = np.empty(N, dtype=np.int64)
    u = lib().orc_bucket_sparse(cone.ctypes.data_as(C.c_void_p), N, keys.ctypes.data_as(C.c_void_p),
                                off.ctypes.data_as(C.c_void_p), perm.ctypes.data_as(C.c_void_p))
    if u < 0:
        raise MemoryError("orc_bucket_sparse")
    return {"top": top, "sign": sg, "cone": cone, "keys": keys[:u].copy(), "offsets": off[:u + 1].copy(),
            "perm": perm, "n_cones": num_cones(X.shape[1], G), "K": X.shape[1], "G": G, "sparse": True}


def search_sparse(X, index, Y, B: int, cones: bool = False, nthreads: int = 0):
    """Algorithm 1 on a sparse table: ``(idx, d32, d64, ncand)`` per query."""
    X, px, xdt = _rows(X)
    Y, py, ydt = _rows(Y)
    N, K = X.shape
    Q = Y.shape[0]
    keys, pk = _arr(index["keys"], np.int64)
    off, po = _arr(index["offsets"], np.int64)
    perm, pp = _arr(index["perm"], np.int64)
    idx = np.empty(Q, dtype=np.int64)
    d32 = np.empty(Q, dtype=np.float32)
    d64 = np.empty(Q, dtype=np.float64)
    nca = np.empty(Q, dtype=np.int64)
    rc = lib().orc_search_sparse(px, xdt, N, K, index["G"], pk, keys.shape[0], po, pp, py, ydt, Q, int(B),
                                 int(bool(cones)), idx.ctypes.data_as(C.c_void_p), d32.ctypes.data_as(C.c_void_p),
                                 d64.ctypes.data_as(C.c_void_p), nca.ctypes.data_as(C.c_void_p), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_search_sparse failed ({rc})")
    return idx, d32, d64, nca

