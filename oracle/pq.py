"""Product quantisation for the oracle (test infrastructure only).

The paper compresses each d-dimensional vector by splitting the dimensions
into m contiguous subspaces and running k-means with 256 centroids in each;
a vector is stored as its m centroid ids (section "Construction of
PQDistTable", first paragraphs of section "BANG").  The paper leaves the
k-means details to the indexing tool; this oracle reads them as:

* training sample: min(n, pq_sample) points drawn without replacement;
* init: 256 distinct sample points per subspace;
* Lloyd iterations in FP64 (nearest centroid by direct squared difference,
  ties to the lowest id; new centroid = mean of its points; an empty
  cluster keeps its previous centroid); stored as FP32;
* no centring, no rotation.
"""
from __future__ import annotations

import ctypes

import numpy as np


def _lib():
    from . import lib
    return lib()


def kmeans_assign(X: np.ndarray, C: np.ndarray, nthreads: int = 0):
    """Lloyd assignment step (FP64).  Returns (assign int32[n], objective)."""
    from . import default_threads
    X = np.ascontiguousarray(X, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    n, ds = X.shape
    K = C.shape[0]
    a = np.empty(n, dtype=np.int32)
    obj = _lib().or_kmeans_assign(X.ctypes.data_as(ctypes.c_void_p), n, ds,
                                  C.ctypes.data_as(ctypes.c_void_p), K,
                                  a.ctypes.data_as(ctypes.c_void_p),
                                  nthreads or default_threads())
    return a, float(obj)


def kmeans(X: np.ndarray, K: int, iters: int, rng, nthreads: int = 0,
           history: list | None = None) -> np.ndarray:
    """Lloyd's k-means on the rows of X (FP64).  `history`, when given,
    receives the objective after each assignment step."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    if n < K:
        raise ValueError(f"k-means needs at least {K} points, got {n}")
    C = X[rng.choice(n, K, replace=False)].copy()
    for _ in range(iters):
        a, obj = kmeans_assign(X, C, nthreads)
        if history is not None:
            history.append(obj)
        cnt = np.bincount(a, minlength=K)
        for t in range(X.shape[1]):
            s = np.bincount(a, weights=X[:, t], minlength=K)
            nz = cnt > 0
            C[nz, t] = s[nz] / cnt[nz]
    return C


def train_pq(sample: np.ndarray, m: int, iters: int, rng,
             nthreads: int = 0) -> np.ndarray:
    """Codebooks cb[m][256][d/m] (FP32) from the training sample."""
    sample = np.asarray(sample)
    n, d = sample.shape
    if d % m:
        raise ValueError("m must divide d")
    ds = d // m
    cb = np.empty((m, 256, ds), dtype=np.float32)
    for j in range(m):
        Xj = sample[:, j * ds:(j + 1) * ds].astype(np.float64)
        cb[j] = kmeans(Xj, 256, iters, rng, nthreads).astype(np.float32)
    return cb


def pq_encode(X: np.ndarray, codebooks: np.ndarray, nthreads: int = 0,
              chunk: int = 1 << 18) -> np.ndarray:
    """codes[n][m] = nearest centroid id per subspace (FP64, ties low)."""
    from . import DT, _dtname, default_threads
    X = np.ascontiguousarray(X)
    cb = np.ascontiguousarray(codebooks, dtype=np.float32)
    n, d = X.shape
    m = cb.shape[0]
    codes = np.empty((n, m), dtype=np.uint8)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        xs = np.ascontiguousarray(X[s:e])
        out = codes[s:e]
        _lib().or_pq_encode(xs.ctypes.data_as(ctypes.c_void_p),
                            DT[_dtname(xs)], e - s, d,
                            cb.ctypes.data_as(ctypes.c_void_p), m,
                            out.ctypes.data_as(ctypes.c_void_p),
                            nthreads or default_threads())
    return codes
