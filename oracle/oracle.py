"""CPU oracle for the TaCo query stage -- TEST INFRASTRUCTURE ONLY.

Defines the expected results the GPU path is checked against.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it; the
product never imports it, and it imports nothing from the product.  Its
inputs come from ``synthdata`` (random draws only).

What lives where:
  * ``taco_oracle.c`` (loaded here through ctypes): the FP32 canonical
    transform and half distances, k-means (Alg 3's clustering step), the
    index file writer/reader, SC-Linear (the index-free baseline of Section
    2.3), Scalable Dynamic Activation (Alg 4) as the
    cell order it produces, Query-aware Candidates Selection (Alg 5) as the
    highest level that exceeds the re-rank budget, the k-ANNS query
    (Alg 6), and FP64 brute-force k-NN (Definition 2).
  * this file: the FP64 statistics of Alg 1 (mean, sample covariance,
    spectral decomposition through LAPACK's symmetric eigensolver), the greedy
    Eigensystem Allocation of Alg 2, the IMI cell lists of Alg 3, and the
    glue that runs the whole index build and writes the index file.

Readings taken where the paper is silent are stated at each function.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

RULE_PRINTED = 0
RULE_PROSE = 1
RULE_FIXED = 2  # SuCo's fixed budget: the floor(beta*n) highest SC-scores, ties by id

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")

_lib_handle = None


class _Dump(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in (
        "qt", "cdist", "corder", "cells", "ncells", "retrieved", "sc", "hist",
        "last", "cand", "ncand", "cand_d32", "cand_d64")]


def lib():
    """The compiled oracle (built on first use if absent)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB):
            from . import build as _b  # noqa: WPS433 (local import: test infra)
            _b.build()
        L = C.CDLL(LIB)
        L.orc_transform.argtypes = [_f32p, C.c_int64, C.c_int, _f32p, _f32p, C.c_int, _f32p]
        L.orc_half_dists.argtypes = [_f32p, _f32p, C.c_int, C.c_int, _f32p]
        L.orc_kmeans.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 _i64p, C.c_void_p, C.c_int64, _f32p, _i32p]
        L.orc_kmeans.restype = C.c_int
        L.orc_write_index.argtypes = [C.c_char_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_uint64, _f32p, _f32p, _f32p, _f32p, _u64p, _u32p,
                                      C.c_void_p]
        L.orc_write_index.restype = C.c_int
        L.orc_load_index.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.orc_load_index.restype = C.c_int
        L.orc_free_index.argtypes = [C.c_void_p]
        L.orc_index_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _i32p]
        for nm, rt in (("orc_index_offsets", C.POINTER(C.c_uint64)),
                       ("orc_index_ids", C.POINTER(C.c_uint32)),
                       ("orc_index_B", C.POINTER(C.c_float)),
                       ("orc_index_mean", C.POINTER(C.c_float)),
                       ("orc_index_base", C.POINTER(C.c_float))):
            getattr(L, nm).argtypes = [C.c_void_p]
            getattr(L, nm).restype = rt
        L.orc_index_centroids.argtypes = [C.c_void_p, C.c_int]
        L.orc_index_centroids.restype = C.POINTER(C.c_float)
        L.orc_argsort.argtypes = [_f32p, C.c_int, _i32p]
        L.orc_probe.argtypes = [_f32p, _i32p, _f32p, _i32p, C.c_int, _i64p, C.c_int64, _i32p,
                                C.POINTER(C.c_int32)]
        L.orc_probe.restype = C.c_int64
        L.orc_threshold.argtypes = [_i64p, C.c_int, C.c_int64, C.c_int]
        L.orc_threshold.restype = C.c_int
        L.orc_select.argtypes = [_u8p, C.c_int64, C.c_int, C.c_int64, C.c_int, _i64p,
                                 C.POINTER(C.c_int32), _i32p]
        L.orc_select.restype = C.c_int64
        L.orc_query.argtypes = [C.c_void_p, _f32p, C.c_double, C.c_double, C.c_int, C.c_int,
                                _i64p, _f32p, _f64p, C.POINTER(_Dump)]
        L.orc_query.restype = C.c_int
        L.orc_query_batch.argtypes = [C.c_void_p, _f32p, C.c_int64, C.c_double, C.c_void_p,
                                      C.c_double, C.c_int, C.c_int, C.c_int, _i64p, C.c_void_p,
                                      C.c_void_p]
        L.orc_query_batch.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_bruteforce.argtypes = [_f32p, C.c_int64, C.c_int, _f32p, C.c_int64, C.c_int,
                                     _i64p, _f64p]
        L.orc_sclinear.argtypes = [C.c_void_p, _f32p, _f32p, C.c_double, C.c_double, C.c_int, _i64p,
                                   _f32p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_sclinear.restype = C.c_int
        L.orc_sclinear_batch.argtypes = [C.c_void_p, _f32p, _f32p, C.c_int64, C.c_double, C.c_double,
                                         C.c_int, C.c_int, _i64p, C.c_void_p]
        L.orc_sclinear_batch.restype = C.c_int
        _lib_handle = L
    return _lib_handle


def max_threads() -> int:
    return int(lib().orc_max_threads())


# --------------------------------------------------------------------------
# Budgets (Alg 4 stop test, Alg 5 budget), evaluated in IEEE double.
# --------------------------------------------------------------------------

def budget_A(alpha: float, n: int) -> int:
    """Collision budget: retrieval stops once at least alpha*n points are
    retrieved (Alg 4).  Integer form ceil(alpha*n), clamped to [1, n]."""
    return int(min(max(math.ceil(alpha * n), 1), n))


def budget_R(beta: float, n: int) -> int:
    """Re-rank budget beta*n of Alg 5 as an integer: floor(beta*n), clamped.
    For an integer x, x <= beta*n exactly when x <= floor(beta*n)."""
    return int(min(max(math.floor(beta * n), 0), n))


# --------------------------------------------------------------------------
# Alg 1: subspace-oriented data transformation (FP64 statistics).
# --------------------------------------------------------------------------

def mean_cov(X: np.ndarray, chunk: int = 1 << 16):
    """Mean and sample covariance 1/(n-1) sum (o-mean)(o-mean)^T in FP64
    (Alg 1, mean and covariance steps).  Sums run over fixed chunks of rows."""
    n, d = X.shape
    s = np.zeros(d, np.float64)
    for lo in range(0, n, chunk):
        s += X[lo:lo + chunk].astype(np.float64).sum(axis=0)
    mean = s / n
    cov = np.zeros((d, d), np.float64)
    for lo in range(0, n, chunk):
        xc = X[lo:lo + chunk].astype(np.float64) - mean
        cov += xc.T @ xc
    cov /= (n - 1)
    return mean, cov


def eigh_desc(cov: np.ndarray):
    """Spectral decomposition (Alg 1) with eigenpairs in descending order.
    Eigenvectors are columns; each is sign-fixed so that its entry of largest
    magnitude (first such on ties) is positive (the paper leaves sign open)."""
    w, v = np.linalg.eigh(cov)
    order = np.argsort(-w, kind="stable")
    w, v = w[order], v[:, order]
    piv = np.argmax(np.abs(v), axis=0)
    sgn = np.sign(v[piv, np.arange(v.shape[1])])
    sgn[sgn == 0] = 1.0
    return w, v * sgn[None, :]


def eigensystem_allocation(evals: np.ndarray, Ns: int, s: int) -> List[List[int]]:
    """Alg 2: deal the top Ns*s eigenpairs into Ns buckets of s.

    Eigenvalues are first scaled by 1/lambda_min over all d of them so that
    every one is >= 1 (values are floored at 1e-12*lambda_max first, which
    guards a singular covariance).  Taking eigenpairs in descending order,
    each goes to the bucket with the smallest product among buckets holding
    fewer than s (ties -> lowest bucket).  Products are compared as sums of
    logs in FP64, which orders them the same way without overflow.  Returns,
    per bucket, the indices (into the descending order) in append order.
    """
    lam = np.asarray(evals, np.float64)
    assert lam.ndim == 1 and Ns * s <= lam.size
    lam = np.maximum(lam, 1e-12 * float(np.max(lam)))
    lam = lam / float(np.min(lam))
    order = np.argsort(-lam, kind="stable")
    logp = [0.0] * Ns
    buckets: List[List[int]] = [[] for _ in range(Ns)]
    for i in range(Ns * s):
        e = int(order[i])
        best = -1
        for j in range(Ns):
            if len(buckets[j]) < s and (best < 0 or logp[j] < logp[best]):
                best = j
        buckets[best].append(e)
        logp[best] += math.log(lam[e])
    return buckets


def transform(X: np.ndarray, mean32: np.ndarray, B32: np.ndarray) -> np.ndarray:
    """r = B^T (o - mean) for every row, canonical FP32 chain (Alg 1)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    M = B32.shape[1]
    T = np.empty((n, M), np.float32)
    lib().orc_transform(X, n, d, np.ascontiguousarray(mean32, np.float32),
                        np.ascontiguousarray(B32, np.float32), M, T)
    return T


# --------------------------------------------------------------------------
# Alg 3: create index.
# --------------------------------------------------------------------------

def kmeans(T: np.ndarray, off: int, h: int, l: int, iters: int, init: np.ndarray,
           train_idx: Optional[np.ndarray] = None):
    """k-means on columns [off, off+h) of T; returns (centroids f32 (l,h),
    final assignment of every row).  See orc_kmeans for the exact rules."""
    T = np.ascontiguousarray(T, np.float32)
    n, ld = T.shape
    cent = np.empty((l, h), np.float32)
    assign = np.empty(n, np.int32)
    init = np.ascontiguousarray(init, np.int64)
    tr = None if train_idx is None else np.ascontiguousarray(train_idx, np.int64)
    n_train = n if tr is None else tr.size
    rc = lib().orc_kmeans(T.ctypes.data, n, ld, off, h, l, iters, init,
                          None if tr is None else tr.ctypes.data, n_train, cent, assign)
    if rc != 0:
        raise RuntimeError(f"orc_kmeans failed ({rc})")
    return cent, assign


def build_imi(a1: np.ndarray, a2: np.ndarray, l: int):
    """IMI of one subspace (Alg 3): point j goes to cell (a1[j], a2[j]),
    stored as cell a1*l + a2; ids are appended for j = 0..n-1, so every cell
    lists its ids ascending.  Returns CSR offsets (l*l+1) and ids (n)."""
    cell = a1.astype(np.int64) * l + a2.astype(np.int64)
    ids = np.argsort(cell, kind="stable").astype(np.uint32)
    counts = np.bincount(cell, minlength=l * l)
    offsets = np.zeros(l * l + 1, np.uint64)
    offsets[1:] = np.cumsum(counts)
    return offsets, ids


def build_index(X: np.ndarray, Ns: int, s: int, l: int, iters: int, init: np.ndarray,
                path: str, train_idx: Optional[np.ndarray] = None, seed: int = 0) -> Dict:
    """Alg 1 + Alg 2 + Alg 3 on base X, written to ``path``.

    Subspace j is transformed columns [j*s, (j+1)*s); its first half is the
    first floor(s/2) of them (each bucket keeps Alg 2's append order, so the
    first half holds its larger-eigenvalue directions), the second half the
    rest.  ``init[j, h]`` are the Forgy seeds (positions into the training
    sample) of half h of subspace j.
    """
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    assert Ns * s <= d and s >= 2
    h1, h2 = s // 2, s - s // 2
    mean64, cov = mean_cov(X)
    evals, evecs = eigh_desc(cov)
    buckets = eigensystem_allocation(evals, Ns, s)
    cols = [e for b in buckets for e in b]
    B32 = np.ascontiguousarray(evecs[:, cols], np.float32)
    mean32 = mean64.astype(np.float32)
    T = transform(X, mean32, B32)
    C1 = np.empty((Ns, l, h1), np.float32)
    C2 = np.empty((Ns, l, h2), np.float32)
    K = l * l
    offsets = np.empty((Ns, K + 1), np.uint64)
    ids = np.empty((Ns, n), np.uint32)
    for j in range(Ns):
        C1[j], a1 = kmeans(T, j * s, h1, l, iters, init[j, 0], train_idx)
        C2[j], a2 = kmeans(T, j * s + h1, h2, l, iters, init[j, 1], train_idx)
        offsets[j], ids[j] = build_imi(a1, a2, l)
    del T
    rc = lib().orc_write_index(path.encode(), n, d, Ns, s, l, seed & (2**64 - 1), mean32, B32,
                               C1, C2, offsets, ids, X.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_write_index failed ({rc})")
    return dict(mean64=mean64, cov=cov, evals=evals, evecs=evecs, buckets=buckets, B32=B32,
                mean32=mean32, C1=C1, C2=C2, offsets=offsets, ids=ids)


def build_workload_index(w, path: str, X: Optional[np.ndarray] = None) -> Dict:
    """Build the index of a ``synthdata`` workload (its seeded base and
    k-means seeding) into ``path``."""
    import synthdata
    if X is None:
        X, _ = synthdata.base_and_queries(w, nq=0)
    train_idx, init = synthdata.kmeans_seeding(w)
    return build_index(X, w.Ns, w.s, w.l, w.iters, init, path, train_idx, w.seed)


# --------------------------------------------------------------------------
# Query side (Alg 4, 5, 6) and ground truth.
# --------------------------------------------------------------------------

def half_dists(x: np.ndarray, cent: np.ndarray) -> np.ndarray:
    cent = np.ascontiguousarray(cent, np.float32)
    l, h = cent.shape
    D = np.empty(l, np.float32)
    lib().orc_half_dists(np.ascontiguousarray(x, np.float32), cent, l, h, D)
    return D


def argsort(D: np.ndarray) -> np.ndarray:
    D = np.ascontiguousarray(D, np.float32)
    idx = np.empty(D.size, np.int32)
    lib().orc_argsort(D, D.size, idx)
    return idx


def probe(D1, idx1, D2, idx2, sizes, A):
    """Alg 4 on one subspace: returns (cells in retrieval order, retrieved).
    ``sizes`` are the l*l cell sizes (cell a*l+b).  See orc_probe for the
    order the cells are taken in."""
    l = len(D1)
    sizes = np.ascontiguousarray(sizes, np.int64)
    assert sizes.size == l * l and 0 < A <= int(sizes.sum())
    cells = np.empty(l * l, np.int32)
    nc = C.c_int32(0)
    got = lib().orc_probe(np.ascontiguousarray(D1, np.float32), np.ascontiguousarray(idx1, np.int32),
            np.ascontiguousarray(D2, np.float32), np.ascontiguousarray(idx2, np.int32),
            l, sizes, int(A), cells, C.byref(nc))
    return cells[:nc.value].copy(), int(got)


def threshold(hist, Ns: int, R: int, rule: int = RULE_PRINTED) -> int:
    return int(lib().orc_threshold(np.ascontiguousarray(hist, np.int64), Ns, int(R), rule))


def select(sc: np.ndarray, Ns: int, R: int, rule: int = RULE_PRINTED):
    """Alg 5: returns (hist, last_collision, candidates ascending)."""
    sc = np.ascontiguousarray(sc, np.uint8)
    hist = np.empty(Ns + 1, np.int64)
    cand = np.empty(sc.size, np.int32)
    last = C.c_int32(0)
    nc = lib().orc_select(sc, sc.size, Ns, int(R), rule, hist, C.byref(last), cand)
    if nc < 0:
        raise MemoryError("orc_select")
    return hist, int(last.value), cand[:nc].copy()


def bruteforce(X: np.ndarray, Q: np.ndarray, k: int):
    """Exact k-NN in FP64: (ids (nq,k) int64, squared distances (nq,k))."""
    X = np.ascontiguousarray(X, np.float32)
    Q = np.ascontiguousarray(Q, np.float32).reshape(-1, X.shape[1])
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.int64)
    dist = np.empty((nq, k), np.float64)
    lib().orc_bruteforce(X, X.shape[0], X.shape[1], Q, nq, k, ids, dist)
    return ids, dist


class OracleIndex:
    """An index file loaded by the oracle's own reader."""

    def __init__(self, path: str):
        h = C.c_void_p()
        rc = lib().orc_load_index(path.encode(), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"orc_load_index({path}) failed ({rc})")
        self._h = h
        n = C.c_int64()
        dims = np.empty(6, np.int32)
        lib().orc_index_info(h, C.byref(n), dims)
        self.n = int(n.value)
        self.d, self.Ns, self.s, self.h1, self.h2, self.l = (int(v) for v in dims)
        self.M = self.Ns * self.s
        self.K = self.l * self.l

    def close(self):
        if self._h:
            lib().orc_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _view(self, ptr, count, dtype):
        return np.ctypeslib.as_array(ptr, shape=(count,)).view(dtype)

    def offsets(self):
        return self._view(lib().orc_index_offsets(self._h), self.Ns * (self.K + 1),
                          np.uint64).reshape(self.Ns, self.K + 1)

    def ids(self):
        return self._view(lib().orc_index_ids(self._h), self.Ns * self.n,
                          np.uint32).reshape(self.Ns, self.n)

    def centroids(self, half: int):
        hh = self.h2 if half else self.h1
        return self._view(lib().orc_index_centroids(self._h, half), self.Ns * self.l * hh,
                          np.float32).reshape(self.Ns, self.l, hh)

    def B(self):
        return self._view(lib().orc_index_B(self._h), self.d * self.M,
                          np.float32).reshape(self.d, self.M)

    def mean(self):
        return self._view(lib().orc_index_mean(self._h), self.d, np.float32)

    def base(self):
        return self._view(lib().orc_index_base(self._h), self.n * self.d,
                          np.float32).reshape(self.n, self.d)

    def query(self, q: np.ndarray, alpha: float, beta: float, k: int,
              rule: int = RULE_PRINTED, dump: bool = True) -> Dict[str, np.ndarray]:
        """Alg 6 on one query; with ``dump`` also every stage's output."""
        q = np.ascontiguousarray(q, np.float32).reshape(self.d)
        ids = np.empty(k, np.int64)
        d32 = np.empty(k, np.float32)
        d64 = np.empty(k, np.float64)
        out = dict(ids=ids, d32=d32, d64=d64)
        dp = None
        if dump:
            Ns, l, K, n = self.Ns, self.l, self.K, self.n
            out.update(
                qt=np.empty(self.M, np.float32), cdist=np.empty((Ns, 2, l), np.float32),
                corder=np.empty((Ns, 2, l), np.int32), cells=np.full((Ns, K), -1, np.int32),
                ncells=np.empty(Ns, np.int32), retrieved=np.empty(Ns, np.int64),
                sc=np.empty(n, np.uint8), hist=np.empty(Ns + 1, np.int64),
                last=np.empty(1, np.int32), cand=np.empty(n, np.int32),
                ncand=np.empty(1, np.int64), cand_d32=np.empty(n, np.float32),
                cand_d64=np.empty(n, np.float64))
            dp = _Dump(*[out[f].ctypes.data for f, _ in _Dump._fields_])
        rc = lib().orc_query(self._h, q, float(alpha), float(beta), int(k), int(rule), ids, d32,
                             d64, C.byref(dp) if dp is not None else None)
        if rc != 0:
            raise ValueError(f"orc_query rejected its arguments ({rc})")
        if dump:
            nc = int(out["ncand"][0])
            out["last"] = int(out["last"][0])
            out["ncand"] = nc
            out["cand"] = out["cand"][:nc]
            out["cand_d32"] = out["cand_d32"][:nc]
            out["cand_d64"] = out["cand_d64"][:nc]
            out["cells"] = [out["cells"][j, :out["ncells"][j]].copy() for j in range(self.Ns)]
        return out

    def transformed_base(self) -> np.ndarray:
        """Every base row transformed with the canonical chain (n x M)."""
        return transform(self.base(), self.mean(), self.B())

    def sclinear(self, T: np.ndarray, q: np.ndarray, alpha: float, beta: float, k: int):
        """SC-Linear on one query (see orc_sclinear); ``T`` from
        transformed_base().  Returns dict(ids, d32, sc, cand)."""
        q = np.ascontiguousarray(q, np.float32).reshape(self.d)
        ids = np.empty(k, np.int64)
        d32 = np.empty(k, np.float32)
        sc = np.empty(self.n, np.uint8)
        cand = np.empty(self.n, np.int32)
        nc = C.c_int64(0)
        rc = lib().orc_sclinear(self._h, np.ascontiguousarray(T, np.float32), q, float(alpha), float(beta),
                                int(k), ids, d32, sc.ctypes.data, cand.ctypes.data, C.byref(nc))
        if rc != 0:
            raise ValueError(f"orc_sclinear rejected its arguments ({rc})")
        return dict(ids=ids, d32=d32, sc=sc, cand=cand[:nc.value].copy())

    def sclinear_batch(self, T: np.ndarray, Q: np.ndarray, alpha: float, beta: float, k: int,
                       nthreads: int = 0):
        """SC-Linear on many queries (parallel over queries): ids (nq, k), d32."""
        Q = np.ascontiguousarray(Q, np.float32).reshape(-1, self.d)
        ids = np.empty((Q.shape[0], k), np.int64)
        d32 = np.empty((Q.shape[0], k), np.float32)
        rc = lib().orc_sclinear_batch(self._h, np.ascontiguousarray(T, np.float32), Q, Q.shape[0],
                                      float(alpha), float(beta), int(k), int(nthreads), ids, d32.ctypes.data)
        if rc != 0:
            raise ValueError(f"orc_sclinear_batch rejected its arguments ({rc})")
        return ids, d32

    def query_batch(self, Q: np.ndarray, alpha, beta: float, k: int, rule: int = RULE_PRINTED,
                    nthreads: int = 0, with_dists: bool = False):
        """Alg 6 on many queries (parallel over queries).  ``alpha`` is a
        float or a per-query array.  Returns ids (nq,k) [, d32, d64]."""
        Q = np.ascontiguousarray(Q, np.float32).reshape(-1, self.d)
        nq = Q.shape[0]
        ids = np.empty((nq, k), np.int64)
        d32 = np.empty((nq, k), np.float32) if with_dists else None
        d64 = np.empty((nq, k), np.float64) if with_dists else None
        per_q = None
        if not np.isscalar(alpha):
            per_q = np.ascontiguousarray(alpha, np.float64)
            assert per_q.size == nq
        rc = lib().orc_query_batch(
            self._h, Q, nq, 0.0 if per_q is not None else float(alpha),
            None if per_q is None else per_q.ctypes.data, float(beta), int(k), int(rule),
            int(nthreads), ids, None if d32 is None else d32.ctypes.data,
            None if d64 is None else d64.ctypes.data)
        if rc != 0:
            raise ValueError(f"orc_query_batch rejected its arguments ({rc})")
        return (ids, d32, d64) if with_dists else ids


def write_index(path: str, mean32, B32, C1, C2, offsets, ids, base, s: int, l: int, seed: int = 0):
    """Write an index file from its parts (the layout the builder writes)."""
    base = np.ascontiguousarray(base, np.float32)
    n, d = base.shape
    Ns = offsets.shape[0]
    rc = lib().orc_write_index(path.encode(), n, d, Ns, s, l, seed, np.ascontiguousarray(mean32, np.float32),
                               np.ascontiguousarray(B32, np.float32), np.ascontiguousarray(C1, np.float32),
                               np.ascontiguousarray(C2, np.float32), np.ascontiguousarray(offsets, np.uint64),
                               np.ascontiguousarray(ids, np.uint32), base.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_write_index failed ({rc})")


def recall_at_k(ids: np.ndarray, gt_d64: np.ndarray, X: np.ndarray, Q: np.ndarray, k: int) -> float:
    """Mean recall |R cap R*|/k (Section 5.1), tie-aware: a returned id
    counts as a true neighbour when its FP64 distance is at most that of the
    k-th true neighbour (exact ties make R* not unique)."""
    nq = ids.shape[0]
    hits = 0
    for i in range(nq):
        r = ids[i, :k]
        r = r[r >= 0]
        if r.size == 0:
            continue
        dd = ((X[r].astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(axis=1)
        hits += int(np.count_nonzero(dd <= gt_d64[i, k - 1]))
    return hits / float(nq * k)
