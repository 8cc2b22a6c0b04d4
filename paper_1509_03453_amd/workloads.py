"""Seeded synthetic workloads for the order-statistics ANN search.

This module only draws random inputs; it holds none of the search method's
arithmetic (no hashing, bucketing, probing or distances), so that the CPU
oracle and the GPU path can be fed the very same arrays without sharing any
code.  Every generator uses numpy's PCG64 (``numpy.random.default_rng``)
with a fixed seed per array.

Workloads (shapes and distributions of the paper's experiments):

* ``gaussian``   i.i.d. N(0,1) FP32 vectors: the paper's running example of
  unstructured data (Section 2 and Section 4.A).  Used with D=16 / N=16384
  (L=1) and with D=64 / N=1e6 (L=2).
* ``descriptor`` 128-D non-negative, heavy-tailed integer components stored
  as uint8 (``rint(min(255, 40*Gamma(0.6,1)))``); queries are database rows
  plus N(0, 8^2) noise clipped to [0, 255].  A synthetic stand-in for the
  128-D SIFT descriptor sets of Section 4.B (the real sets are not used).
* ``patches``    mean-removed 8x8 patches (D=64, FP16) at every pixel of a
  2048x2048 Gaussian field with a 1/f amplitude spectrum; queries are the
  patches of the same field shifted by (3,5) plus N(0, 0.05^2) noise.  A
  stand-in for the nearest-neighbour field of the copy-move application of
  Section 4.C (the real images are not used).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian_db", "gaussian_queries", "descriptor_db", "descriptor_queries",
    "patch_field", "patch_rows", "patch_pair", "serving_requests",
    "tie_heavy", "random_bases", "random_signs", "SEEDS",
]

# One seed per array, 1000*workload + k.
SEEDS = {
    "gauss16_db": 1001, "gauss16_q": 1002,
    "gauss64_db": 2001, "gauss64_q": 2002,
    "desc_db": 3001, "desc_pick": 3002, "desc_noise": 3003,
    "sift_db": 3011, "kmeans_init": 3012,
    "patch_field": 4001, "patch_noise": 4002, "patch_sample": 4003,
    "serve_arrivals": 5001,
    "bases": 6001, "wht_signs": 6002,
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def gaussian_db(n: int, d: int, seed: int) -> np.ndarray:
    """``n x d`` i.i.d. standard normal rows, FP32, row-major."""
    return _rng(seed).standard_normal((int(n), int(d)), dtype=np.float32)


def gaussian_queries(q: int, d: int, seed: int) -> np.ndarray:
    """Queries drawn from the same source as the database (own seed)."""
    return _rng(seed).standard_normal((int(q), int(d)), dtype=np.float32)


def descriptor_db(n: int, d: int = 128, seed: int = SEEDS["desc_db"]) -> np.ndarray:
    """uint8 rows ``rint(min(255, 40*G))`` with ``G ~ Gamma(shape 0.6, scale 1)``."""
    g = _rng(seed).gamma(0.6, 1.0, size=(int(n), int(d)))
    return np.rint(np.minimum(255.0, 40.0 * g)).astype(np.uint8)


def sift_like_db(n: int, d: int = 128, seed: int = SEEDS["sift_db"], decay: float = 1.1,
                 scale: float = 130.0, mean: float = 40.0) -> np.ndarray:
    """uint8 rows with strongly correlated components, a stand-in for the SIFT
    descriptors of Section 4.B: ``rint(clip(mean + A z, 0, 255))`` with ``A`` a
    seeded Haar-random orthonormal ``d x d`` matrix and independent
    ``z_i ~ N(0, scale^2 i^-decay)`` (i = 1..d), so that the first 16
    principal components hold about 70% of the energy (the share the paper
    reports for its SIFT sets)."""
    r = _rng(seed)
    a = r.standard_normal((int(d), int(d)))
    q, rr = np.linalg.qr(a)
    q = q * np.sign(np.diag(rr))[None, :]
    sig = scale * np.arange(1, int(d) + 1, dtype=np.float64) ** (-decay / 2.0)
    out = np.empty((int(n), int(d)), dtype=np.uint8)
    chunk = 1 << 16
    for s in range(0, int(n), chunk):
        m = min(chunk, int(n) - s)
        z = r.standard_normal((m, int(d))) * sig[None, :]
        out[s:s + m] = np.rint(np.clip(mean + z @ q.T, 0.0, 255.0)).astype(np.uint8)
    return out


def pick_rows(n: int, k: int, seed: int = SEEDS["kmeans_init"]) -> np.ndarray:
    """``k`` distinct row ids out of ``n`` in increasing order (seeded), e.g.
    the initial k-means centroids."""
    return np.sort(_rng(seed).choice(int(n), size=int(k), replace=False))


def descriptor_queries(db_u8: np.ndarray, q: int,
                       pick_seed: int = SEEDS["desc_pick"],
                       noise_seed: int = SEEDS["desc_noise"]) -> tuple[np.ndarray, np.ndarray]:
    """Queries = picked database rows + N(0, 8^2), clipped to [0, 255], FP32.

    Returns ``(queries_f32, source_rows)``; ``source_rows`` are the picked
    row ids (the true neighbour almost always)."""
    n, d = db_u8.shape
    src = _rng(pick_seed).integers(0, n, size=int(q), dtype=np.int64)
    noise = _rng(noise_seed).normal(0.0, 8.0, size=(int(q), d))
    y = np.clip(db_u8[src].astype(np.float64) + noise, 0.0, 255.0)
    return y.astype(np.float32), src


def patch_field(size: int = 2048, seed: int = SEEDS["patch_field"]) -> np.ndarray:
    """Zero-mean, unit-std Gaussian field with amplitude spectrum 1/|f|.

    ``F = Re(ifft2(fft2(w) * A))``, ``w ~ N(0,1)``, ``A(f) = 1/|f|`` and
    ``A(0) = 0``.  Returned as float64 ``size x size``."""
    w = _rng(seed).standard_normal((size, size))
    fy = np.fft.fftfreq(size)[:, None]
    fx = np.fft.fftfreq(size)[None, :]
    r = np.sqrt(fx * fx + fy * fy)
    amp = np.zeros_like(r)
    amp[r > 0] = 1.0 / r[r > 0]
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
    f -= f.mean()
    f /= f.std()
    return f


def patch_rows(img: np.ndarray, p: int = 8, rows: np.ndarray | None = None) -> np.ndarray:
    """Mean-removed ``p x p`` patches (row-major, FP16) at every valid top-left.

    The mean is removed in FP32 and the result rounded to FP16 (round to
    nearest even).  ``rows`` optionally selects patch ids (``r*W + c`` with
    ``W = size - p + 1``) instead of all of them."""
    win = np.lib.stride_tricks.sliding_window_view(img.astype(np.float32), (p, p))
    hh, ww = win.shape[:2]
    flat = win.reshape(hh * ww, p * p)
    if rows is not None:
        flat = flat[np.asarray(rows, dtype=np.int64)]
    out = np.empty(flat.shape, dtype=np.float16)
    chunk = 1 << 18
    for s in range(0, flat.shape[0], chunk):
        blk = np.ascontiguousarray(flat[s:s + chunk], dtype=np.float32)
        blk = blk - blk.mean(axis=1, keepdims=True, dtype=np.float32)
        out[s:s + chunk] = blk.astype(np.float16)
    return out


def patch_pair(size: int = 2048, p: int = 8, shift=(3, 5), noise: float = 0.05,
               field_seed: int = SEEDS["patch_field"],
               noise_seed: int = SEEDS["patch_noise"]) -> tuple[np.ndarray, np.ndarray]:
    """Database patches of the field and query patches of the shifted, noisy field."""
    f = patch_field(size, field_seed)
    g = np.roll(f, shift, axis=(0, 1)) + _rng(noise_seed).normal(0.0, noise, size=f.shape)
    return patch_rows(f, p), patch_rows(g, p)


def tie_heavy(n: int, d: int, seed: int, values=(-2, -1, 0, 1, 2),
              neg_zero: bool = True) -> np.ndarray:
    """Small-integer FP32 rows (many |x| ties) with some zeros stored as -0.0."""
    r = _rng(seed)
    x = r.choice(np.asarray(values, dtype=np.float32), size=(int(n), int(d)))
    if neg_zero:
        flip = (x == 0) & (r.random(size=x.shape) < 0.5)
        x[flip] = np.float32(-0.0)
    return x


def serving_requests(n_req: int, rate: float, n_indexes: int, max_q: int = 4096,
                     seed: int = SEEDS["serve_arrivals"]):
    """Poisson arrivals: ``(arrival_s, index_id, n_queries, query_seed)`` rows.

    Inter-arrival times ~ Exp(1/rate); index uniform over ``n_indexes``;
    batch size uniform in 1..max_q; each request gets its own query seed."""
    r = _rng(seed)
    gaps = r.exponential(1.0 / float(rate), size=int(n_req))
    t = np.cumsum(gaps)
    which = r.integers(0, n_indexes, size=int(n_req))
    sizes = r.integers(1, int(max_q) + 1, size=int(n_req))
    qseeds = r.integers(1 << 20, 1 << 30, size=int(n_req))
    return [(float(a), int(b), int(c), int(s)) for a, b, c, s in zip(t, which, sizes, qseeds)]


def random_bases(n: int, d: int, seed: int = SEEDS["bases"], identity_first: bool = True) -> np.ndarray:
    """``n`` orthonormal ``d x d`` FP32 matrices, row-major, for the
    several-bases search: the Q factor of a Gaussian matrix with the signs of
    R's diagonal folded in (Haar-distributed), in float64 then rounded.  The
    first one is the identity when ``identity_first`` (the original basis)."""
    r = _rng(seed)
    out = np.empty((int(n), int(d), int(d)), dtype=np.float32)
    for k in range(int(n)):
        if k == 0 and identity_first:
            out[k] = np.eye(d, dtype=np.float32)
            continue
        a = r.standard_normal((d, d))
        q, rr = np.linalg.qr(a)
        q = q * np.sign(np.diag(rr))[None, :]
        out[k] = q.astype(np.float32)
    return out


def random_signs(n: int, d: int, seed: int = SEEDS["wht_signs"]) -> np.ndarray:
    """``n`` vectors of ``d`` independent fair signs (+1.0 / -1.0, FP32): the
    diagonal of the structured bases H diag(s)."""
    return np.where(_rng(seed).random((int(n), int(d))) < 0.5, -1.0, 1.0).astype(np.float32)



def prototype_rows(n_proto: int, per: int, d: int, n_big: int, noise: float = 0.3,
                   seed: int = 7301) -> np.ndarray:
    """Clustered FP32 rows: ``n_proto`` prototypes, each with ``n_big``
    components of magnitude 8..12 (random indices and signs) over N(0, 0.5^2)
    background, and ``per`` copies of each plus N(0, noise^2).  Copies of one
    prototype mostly share their largest components, so a table with very
    many cones still has populated neighbourhoods."""
    r = _rng(seed)
    protos = r.normal(0.0, 0.5, size=(n_proto, d))
    for p in range(n_proto):
        idx = r.choice(d, size=n_big, replace=False)
        protos[p, idx] = r.uniform(8.0, 12.0, size=n_big) * r.choice([-1.0, 1.0], size=n_big)
    rows = np.repeat(protos, per, axis=0) + r.normal(0.0, noise, size=(n_proto * per, d))
    return rows.astype(np.float32)
