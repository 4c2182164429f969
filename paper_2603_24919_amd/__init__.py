"""Python binding of ``libtaco_hip.so``, the gfx950 query stage of TaCo.

Argument marshalling only: every step of a search runs in the library's HIP
kernels.  Functions carry the C-ABI's names (``include/taco.h``); tensors
are torch CUDA tensors used as device memory, and the default stream is
torch's current stream on the index's device.  Importing the package does
not touch the GPU; the first call loads the library and raises
``TacoLibraryMissing`` if it has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Tuple

import numpy as np

__all__ = [
    "TC_OK", "TC_EINVAL", "TC_EIO", "TC_EFORMAT", "TC_ENOMEM", "TC_EDEVICE",
    "TC_RULE_PRINTED", "TC_RULE_PROSE", "TC_RULE_FIXED", "TC_OPT_SELECT_RULE", "TC_OPT_MAX_BATCH",
    "TC_OPT_TILE_IDS", "TC_OPT_PROFILE", "TC_OPT_SCRATCH_BYTES", "TC_OPT_PRECISION",
    "TC_FP32", "TC_BF16", "TC_OPT_COUNT_MODE", "TC_COUNT_AUTO", "TC_COUNT_SPLIT",
    "TC_COUNT_FUSED", "TC_COUNT_LIST", "TC_COUNT_CODES", "TC_OPT_LIST_LEVEL", "TC_OPT_GRAPH", "TC_OPT_PROBE_QPW", "TC_OPT_RERANK_BLOCKS", "KERNELS",
    "TC_OPT_CDIST_PRECISION", "TC_CDIST_FP32", "TC_CDIST_BF16", "TC_CDIST_FP8", "TC_U8",
    "tc_device_errors", "tc_search_batched", "tc_autotune", "tc_autotune_batched", "tc_search_noalloc",
    "tc_search_sclinear",
    "TC_OPT_TUNE_PRECISION", "TC_OPT_COUNT_QPW", "TC_OPT_CANDIDATE_SLOTS", "TC_OPT_COUNT_BLOCK",
    "TacoError", "TacoLibraryMissing", "lib_path", "load_library",
    "tc_load_index", "tc_free_index", "tc_index_info", "tc_set_option", "tc_search",
    "tc_search_debug", "tc_kernel_time", "tc_profile_reset", "tc_batch_capacity",
    "tc_last_error", "Index", "DUMP_FIELDS",
]

TC_OK, TC_EINVAL, TC_EIO, TC_EFORMAT, TC_ENOMEM, TC_EDEVICE = 0, -1, -2, -3, -4, -5
TC_RULE_PRINTED, TC_RULE_PROSE, TC_RULE_FIXED = 0, 1, 2
TC_OPT_SELECT_RULE, TC_OPT_MAX_BATCH, TC_OPT_TILE_IDS, TC_OPT_PROFILE, TC_OPT_SCRATCH_BYTES = 1, 2, 3, 4, 5
TC_OPT_PRECISION = 6
TC_FP32, TC_BF16, TC_U8 = 0, 1, 2
TC_OPT_COUNT_MODE = 7
TC_COUNT_AUTO, TC_COUNT_SPLIT, TC_COUNT_FUSED, TC_COUNT_LIST, TC_COUNT_CODES = 0, 1, 2, 3, 4
TC_OPT_LIST_LEVEL = 12
TC_OPT_TUNE_PRECISION = 13
TC_OPT_COUNT_QPW = 14
TC_OPT_CANDIDATE_SLOTS = 15
TC_OPT_COUNT_BLOCK = 16
TC_OPT_GRAPH, TC_OPT_PROBE_QPW, TC_OPT_RERANK_BLOCKS = 8, 9, 10
TC_OPT_CDIST_PRECISION = 11
TC_CDIST_FP32, TC_CDIST_BF16, TC_CDIST_FP8 = 0, 1, 2
KERNELS = ("transform", "probe", "count", "select", "rerank", "topk", "recheck", "count_select",
           "graph", "cdist", "stream")

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libtaco_hip.so"


class TacoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"taco error {code}: {msg}")
        self.code = code


class TacoLibraryMissing(ImportError):
    pass


class _StageDump(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in (
        "qt", "cdist", "corder", "cells", "ncells", "retrieved", "sc", "hist", "last",
        "ncand", "cand", "cand_dist", "nrecheck")]


DUMP_FIELDS = tuple(f for f, _ in _StageDump._fields_)

_lib = None


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load the built library (once).  No fallback: a missing library is an
    error, whether or not a GPU is present."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise TacoLibraryMissing(
            f"{path} is not built; run paper_2603_24919_amd/build.py (or __graft_entry__.build())")
    L = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.tc_load_index.argtypes = [C.c_char_p, C.c_int, C.POINTER(vp)]
    L.tc_free_index.argtypes = [vp]
    L.tc_free_index.restype = None
    L.tc_index_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                C.POINTER(i32), C.POINTER(i32)]
    L.tc_set_option.argtypes = [vp, C.c_int, i64]
    L.tc_search.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, vp, vp]
    L.tc_search_noalloc.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, vp, vp]
    L.tc_search_sclinear.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, vp, vp, C.POINTER(_StageDump)]
    L.tc_search_debug.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, vp, vp, C.POINTER(_StageDump)]
    L.tc_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(dbl), C.POINTER(i64)]
    L.tc_profile_reset.argtypes = [vp]
    L.tc_batch_capacity.argtypes = [vp, dbl, i32, C.POINTER(i64)]
    L.tc_device_errors.argtypes = [vp, C.POINTER(C.c_uint32)]
    L.tc_search_batched.argtypes = [vp, vp, i64, vp, vp, i32, dbl, vp, vp, vp]
    L.tc_autotune.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, C.c_char_p, C.c_char_p, C.c_size_t]
    L.tc_autotune_batched.argtypes = [vp, vp, i64, vp, vp, i32, dbl, vp, C.c_char_p, C.c_char_p,
                                      C.c_size_t]
    L.tc_last_error.restype = C.c_char_p
    L.tc_last_error.argtypes = []
    L.tc_build_stats.argtypes = [vp, i64, i32, vp, vp, vp]
    L.tc_build_eigen.argtypes = [vp, i32, vp, vp, vp]
    L.tc_build_allocate.argtypes = [vp, i32, i32, i32, vp]
    L.tc_build_transform.argtypes = [vp, i64, i32, vp, vp, i32, vp, vp]
    L.tc_build_kmeans.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, i64, vp, vp, vp]
    L.tc_build_imi.argtypes = [vp, i64, i32, i32, vp, vp, vp]
    L.tc_build_index.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, i64, C.c_uint64, vp, vp,
                                 C.c_int, C.POINTER(vp), vp]
    L.tc_save_index.argtypes = [vp, C.c_char_p]
    for f in ("tc_load_index", "tc_index_info", "tc_set_option", "tc_search", "tc_search_noalloc",
              "tc_search_sclinear",
              "tc_search_debug",
              "tc_kernel_time", "tc_profile_reset", "tc_batch_capacity", "tc_device_errors",
              "tc_search_batched", "tc_autotune", "tc_autotune_batched", "tc_build_stats", "tc_build_eigen",
              "tc_build_allocate", "tc_build_transform", "tc_build_kmeans", "tc_build_imi",
              "tc_build_index", "tc_save_index"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def tc_last_error() -> str:
    return load_library().tc_last_error().decode()


def _check(rc: int):
    if rc != TC_OK:
        raise TacoError(rc, tc_last_error())


def tc_load_index(path: str, device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check(load_library().tc_load_index(os.fsencode(path), int(device), C.byref(h)))
    return h


def tc_free_index(index) -> None:
    if index:
        load_library().tc_free_index(index)


def tc_index_info(index) -> Dict[str, int]:
    n, d, Ns, s, l = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load_library().tc_index_info(index, C.byref(n), C.byref(d), C.byref(Ns), C.byref(s),
                                        C.byref(l)))
    return dict(n=n.value, d=d.value, Ns=Ns.value, s=s.value, l=l.value)


def tc_set_option(index, option: int, value: int) -> None:
    _check(load_library().tc_set_option(index, int(option), int(value)))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check_tensor(t, dtype, shape, device, name):
    import torch
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")
    if device is not None and t.device != torch.device(device):
        raise ValueError(f"{name} must live on {device}")


# --------------------------------------------------------------------------
# Index construction (Alg 1-3).  Argument marshalling only: every stage runs
# in the library's kernels (Alg 2 in its host code).
# --------------------------------------------------------------------------

def _host_i64(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


def tc_build_stats(X, stream=None):
    """Alg 1 statistics of ``X`` (CUDA float32 [n, d]): FP64 (mean [d], cov [d, d])."""
    import torch
    n, d = X.shape
    _check_tensor(X, torch.float32, (n, d), None, "X")
    mean = torch.empty(d, dtype=torch.float64, device=X.device)
    cov = torch.empty((d, d), dtype=torch.float64, device=X.device)
    _check(load_library().tc_build_stats(_ptr(X), n, d, _ptr(mean), _ptr(cov),
                                         _stream_handle(stream, X.device)))
    return mean, cov


def tc_build_eigen(cov, stream=None):
    """Alg 1 spectral decomposition of ``cov`` (CUDA float64 [d, d]):
    (evals [d] descending, evecs [d, d] with eigenvectors as columns)."""
    import torch
    d = cov.shape[0]
    _check_tensor(cov, torch.float64, (d, d), None, "cov")
    ev = torch.empty(d, dtype=torch.float64, device=cov.device)
    V = torch.empty((d, d), dtype=torch.float64, device=cov.device)
    _check(load_library().tc_build_eigen(_ptr(cov), d, _ptr(ev), _ptr(V), _stream_handle(stream, cov.device)))
    return ev, V


def tc_build_allocate(evals, Ns: int, s: int) -> np.ndarray:
    """Alg 2 on host eigenvalues (descending): column order, [Ns*s] int32."""
    ev = np.ascontiguousarray(evals, dtype=np.float64)
    cols = np.empty(Ns * s, dtype=np.int32)
    _check(load_library().tc_build_allocate(ev.ctypes.data, ev.size, Ns, s, cols.ctypes.data))
    return cols


def tc_build_transform(X, mean, B, stream=None):
    """T = B^T (X - mean) row by row (CUDA float32 in and out)."""
    import torch
    n, d = X.shape
    M = B.shape[1]
    _check_tensor(X, torch.float32, (n, d), None, "X")
    _check_tensor(mean, torch.float32, (d,), X.device, "mean")
    _check_tensor(B, torch.float32, (d, M), X.device, "B")
    T = torch.empty((n, M), dtype=torch.float32, device=X.device)
    _check(load_library().tc_build_transform(_ptr(X), n, d, _ptr(mean), _ptr(B), M, _ptr(T),
                                             _stream_handle(stream, X.device)))
    return T


def tc_build_kmeans(T, Ns: int, s: int, l: int, iters: int, init, train=None, stream=None):
    """Alg 3 k-means of every half-subspace of ``T`` (CUDA float32 [n, ld]);
    ``init`` host [Ns, 2, l] seed positions, ``train`` host sorted rows or None.
    Returns (cent float32 [2*Ns, l, s - s//2], assign int32 [2*Ns, n])."""
    import torch
    n, ld = T.shape
    _check_tensor(T, torch.float32, (n, ld), None, "T")
    init = _host_i64(init)
    train = _host_i64(train)
    if init.size != 2 * Ns * l:
        raise ValueError("init must hold 2*Ns*l positions")
    cent = torch.empty((2 * Ns, l, s - s // 2), dtype=torch.float32, device=T.device)
    assign = torch.empty((2 * Ns, n), dtype=torch.int32, device=T.device)
    _check(load_library().tc_build_kmeans(
        _ptr(T), n, ld, Ns, s, l, iters, init.ctypes.data,
        None if train is None else train.ctypes.data, 0 if train is None else train.size,
        _ptr(cent), _ptr(assign), _stream_handle(stream, T.device)))
    return cent, assign


def tc_build_imi(assign, Ns: int, l: int, stream=None):
    """Alg 3 IMI from labels (CUDA int32 [2*Ns, n]): (offsets uint32 as int32
    [Ns, l*l+1], ids as int32 [Ns, n])."""
    import torch
    G, n = assign.shape
    _check_tensor(assign, torch.int32, (2 * Ns, n), None, "assign")
    offs = torch.empty((Ns, l * l + 1), dtype=torch.int32, device=assign.device)
    ids = torch.empty((Ns, n), dtype=torch.int32, device=assign.device)
    _check(load_library().tc_build_imi(_ptr(assign), n, Ns, l, _ptr(offs), _ptr(ids),
                                       _stream_handle(stream, assign.device)))
    return offs, ids


def tc_build_index(base, Ns: int, s: int, l: int, iters: int, init, train=None, seed: int = 0,
                   mean=None, B=None, device: int = 0):
    """Alg 1-3 on the GPU from ``base`` (CUDA float32 [n, d]).  Returns
    (index handle, stage milliseconds [statistics, eigensolver, allocation,
    transform, k-means, IMI])."""
    import torch
    n, d = base.shape
    _check_tensor(base, torch.float32, (n, d), device, "base")
    init = _host_i64(init)
    train = _host_i64(train)
    if init.size != 2 * Ns * l:
        raise ValueError("init must hold 2*Ns*l positions")
    if (mean is None) != (B is None):
        raise ValueError("give both mean and B, or neither")
    m32 = None if mean is None else np.ascontiguousarray(mean, dtype=np.float32)
    B32 = None if B is None else np.ascontiguousarray(B, dtype=np.float32)
    ms = np.zeros(6, dtype=np.float64)
    h = C.c_void_p()
    _check(load_library().tc_build_index(
        _ptr(base), n, d, Ns, s, l, iters, init.ctypes.data,
        None if train is None else train.ctypes.data, 0 if train is None else train.size,
        int(seed) & (2**64 - 1), None if m32 is None else m32.ctypes.data,
        None if B32 is None else B32.ctypes.data, int(device), C.byref(h), ms.ctypes.data))
    return h, ms


def tc_save_index(index, path: str) -> None:
    _check(load_library().tc_save_index(index, os.fsencode(path)))


def tc_search(index, queries, k: int, alpha: float, beta: float, ids=None, dists=None,
              stream=None) -> Tuple["object", "object"]:
    """Enqueue a search of ``queries`` (CUDA float32 [nq, d]); returns
    ``(ids int64 [nq, k], dists float32 [nq, k])`` (allocated if not given)."""
    return tc_search_debug(index, queries, k, alpha, beta, None, ids, dists, stream)


def tc_search_noalloc(index, queries, k: int, alpha: float, beta: float, ids, dists,
                      stream=None) -> None:
    """Enqueue the search with no device allocation (tc_search_noalloc) into
    the caller's ``ids`` (CUDA int64 [nq, k]) and ``dists`` (float32)."""
    import torch
    nq = int(queries.shape[0])
    dev = queries.device
    if queries.dtype != torch.float32 or not queries.is_cuda or not queries.is_contiguous():
        raise ValueError("queries must be a contiguous float32 CUDA tensor")
    _check_tensor(ids, torch.int64, (nq, k), dev, "ids")
    _check_tensor(dists, torch.float32, (nq, k), dev, "dists")
    _check(load_library().tc_search_noalloc(index, queries.data_ptr(), nq, int(k), float(alpha),
                                            float(beta), ids.data_ptr(), dists.data_ptr(),
                                            _stream_handle(stream, dev)))


def tc_search_debug(index, queries, k: int, alpha: float, beta: float, dump=None, ids=None,
                    dists=None, stream=None):
    """tc_search plus per-stage outputs into the CUDA tensors of the ``dump``
    dict (keys from ``DUMP_FIELDS``; shapes as in include/taco.h)."""
    import torch
    nq = int(queries.shape[0])
    dev = queries.device
    if ids is None:
        ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    if dists is None:
        dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    if queries.dtype != torch.float32 or not queries.is_cuda or not queries.is_contiguous():
        raise ValueError("queries must be a contiguous float32 CUDA tensor")
    _check_tensor(ids, torch.int64, (nq, k), dev, "ids")
    _check_tensor(dists, torch.float32, (nq, k), dev, "dists")
    st = _stream_handle(stream, dev)
    L = load_library()
    if dump is None:
        rc = L.tc_search(index, queries.data_ptr(), nq, int(k), float(alpha), float(beta),
                         ids.data_ptr(), dists.data_ptr(), st)
    else:
        unknown = set(dump) - set(DUMP_FIELDS)
        if unknown:
            raise ValueError(f"unknown dump fields {sorted(unknown)}")
        for t in dump.values():
            if not (t.is_cuda and t.is_contiguous()):
                raise ValueError("dump tensors must be contiguous CUDA tensors")
        sd = _StageDump(*[_ptr(dump.get(f)) for f in DUMP_FIELDS])
        rc = L.tc_search_debug(index, queries.data_ptr(), nq, int(k), float(alpha), float(beta),
                               ids.data_ptr(), dists.data_ptr(), st, C.byref(sd))
    _check(rc)
    return ids, dists


def tc_search_sclinear(index, queries, k: int, alpha: float, beta: float, dump=None, ids=None,
                       dists=None, stream=None):
    """SC-Linear (the index-free baseline) on ``queries``; ``dump`` as for
    tc_search_debug (sc, hist, last, ncand, cand are written).  Returns
    ``(ids, dists)``."""
    import torch
    nq = int(queries.shape[0])
    dev = queries.device
    if queries.dtype != torch.float32 or not queries.is_cuda or not queries.is_contiguous():
        raise ValueError("queries must be a contiguous float32 CUDA tensor")
    if ids is None:
        ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    if dists is None:
        dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    _check_tensor(ids, torch.int64, (nq, k), dev, "ids")
    _check_tensor(dists, torch.float32, (nq, k), dev, "dists")
    sd = None
    if dump is not None:
        unknown = set(dump) - set(DUMP_FIELDS)
        if unknown:
            raise ValueError(f"unknown dump fields {sorted(unknown)}")
        sd = _StageDump(*[_ptr(dump.get(f)) for f in DUMP_FIELDS])
    _check(load_library().tc_search_sclinear(index, queries.data_ptr(), nq, int(k), float(alpha), float(beta),
                                             ids.data_ptr(), dists.data_ptr(), _stream_handle(stream, dev),
                                             None if sd is None else C.byref(sd)))
    return ids, dists


def tc_search_batched(index, queries, alpha, k, k_max: int, beta: float, ids=None, dists=None,
                      stream=None):
    """Per-query budgets: ``alpha`` (CUDA float64 [nq]) and ``k`` (CUDA int32
    [nq]); returns ``(ids int64 [nq, k_max], dists float32 [nq, k_max])``."""
    import torch
    nq = int(queries.shape[0])
    dev = queries.device
    if queries.dtype != torch.float32 or not queries.is_cuda or not queries.is_contiguous():
        raise ValueError("queries must be a contiguous float32 CUDA tensor")
    _check_tensor(alpha, torch.float64, (nq,), dev, "alpha")
    _check_tensor(k, torch.int32, (nq,), dev, "k")
    if ids is None:
        ids = torch.empty((nq, k_max), dtype=torch.int64, device=dev)
    if dists is None:
        dists = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
    _check_tensor(ids, torch.int64, (nq, k_max), dev, "ids")
    _check_tensor(dists, torch.float32, (nq, k_max), dev, "dists")
    _check(load_library().tc_search_batched(index, queries.data_ptr(), nq, alpha.data_ptr(),
                                            k.data_ptr(), int(k_max), float(beta), ids.data_ptr(),
                                            dists.data_ptr(), _stream_handle(stream, dev)))
    return ids, dists


def tc_autotune(index, queries, k: int, alpha: float, beta: float, cache_path=None, stream=None) -> str:
    """Tune the launch configuration on this batch; returns the report."""
    buf = C.create_string_buffer(8192)
    _check(load_library().tc_autotune(
        index, queries.data_ptr(), int(queries.shape[0]), int(k), float(alpha), float(beta),
        _stream_handle(stream, queries.device), None if cache_path is None else os.fsencode(cache_path),
        buf, len(buf)))
    return buf.value.decode()


def tc_autotune_batched(index, queries, alpha, k, k_max: int, beta: float, cache_path=None,
                        stream=None) -> str:
    """Tune the launch configuration of tc_search_batched on this batch and
    its per-query budgets (CUDA float64 ``alpha`` [nq], int32 ``k`` [nq]);
    returns the report."""
    import torch
    nq = int(queries.shape[0])
    dev = queries.device
    _check_tensor(alpha, torch.float64, (nq,), dev, "alpha")
    _check_tensor(k, torch.int32, (nq,), dev, "k")
    buf = C.create_string_buffer(8192)
    _check(load_library().tc_autotune_batched(
        index, queries.data_ptr(), nq, alpha.data_ptr(), k.data_ptr(), int(k_max), float(beta),
        _stream_handle(stream, dev), None if cache_path is None else os.fsencode(cache_path),
        buf, len(buf)))
    return buf.value.decode()


def tc_kernel_time(index, kernel: str) -> Tuple[float, int]:
    ms, n = C.c_double(), C.c_int64()
    _check(load_library().tc_kernel_time(index, kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def tc_profile_reset(index) -> None:
    _check(load_library().tc_profile_reset(index))


def tc_device_errors(index) -> int:
    v = C.c_uint32()
    _check(load_library().tc_device_errors(index, C.byref(v)))
    return v.value


def tc_batch_capacity(index, beta: float, k_max: int) -> int:
    """Queries per internal batch of a call with re-rank ratio beta and
    k_max results per query."""
    v = C.c_int64()
    _check(load_library().tc_batch_capacity(index, float(beta), int(k_max), C.byref(v)))
    return v.value


class Index:
    """Owning wrapper of a loaded index."""

    def __init__(self, path: Optional[str], device: int = 0, handle=None):
        self.device = int(device)
        self.handle = handle if handle is not None else tc_load_index(path, self.device)
        self.stage_ms = None
        info = tc_index_info(self.handle)
        self.n, self.d, self.Ns, self.s, self.l = (info[x] for x in ("n", "d", "Ns", "s", "l"))
        self.M, self.K = self.Ns * self.s, self.l * self.l

    @classmethod
    def build(cls, base, Ns: int, s: int, l: int, iters: int, init, train=None, seed: int = 0,
              mean=None, B=None, device: int = 0) -> "Index":
        """Index built on the GPU from ``base`` (Alg 1-3); ``stage_ms`` holds the
        stage times of the build."""
        h, ms = tc_build_index(base, Ns, s, l, iters, init, train, seed, mean, B, device)
        idx = cls(None, device, handle=h)
        idx.stage_ms = ms
        return idx

    def save(self, path: str) -> None:
        tc_save_index(self.handle, path)

    def close(self):
        if self.handle:
            tc_free_index(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        tc_set_option(self.handle, option, value)

    def search(self, queries, k: int, alpha: float, beta: float, **kw):
        return tc_search(self.handle, queries, k, alpha, beta, **kw)

    def search_sclinear(self, queries, k: int, alpha: float, beta: float, dump=None, **kw):
        return tc_search_sclinear(self.handle, queries, k, alpha, beta, dump, **kw)

    def search_noalloc(self, queries, k: int, alpha: float, beta: float, ids, dists, **kw):
        return tc_search_noalloc(self.handle, queries, k, alpha, beta, ids, dists, **kw)

    def search_batched(self, queries, alpha, k, k_max: int, beta: float, **kw):
        return tc_search_batched(self.handle, queries, alpha, k, k_max, beta, **kw)

    def autotune(self, queries, k: int, alpha: float, beta: float, cache_path=None, **kw) -> str:
        return tc_autotune(self.handle, queries, k, alpha, beta, cache_path=cache_path, **kw)

    def autotune_batched(self, queries, alpha, k, k_max: int, beta: float, cache_path=None,
                         **kw) -> str:
        return tc_autotune_batched(self.handle, queries, alpha, k, k_max, beta,
                                   cache_path=cache_path, **kw)

    def search_debug(self, queries, k: int, alpha: float, beta: float, dump, **kw):
        return tc_search_debug(self.handle, queries, k, alpha, beta, dump, **kw)

    def dump_buffers(self, nq: int, fields=DUMP_FIELDS):
        """Allocate stage-dump tensors for ``nq`` queries on the index's GPU."""
        import torch
        dev = torch.device("cuda", self.device)
        shapes = dict(
            qt=((nq, self.M), torch.float32), cdist=((nq, self.Ns, 2, self.l), torch.float32),
            corder=((nq, self.Ns, 2, self.l), torch.int32),
            cells=((nq, self.Ns, self.K), torch.int32), ncells=((nq, self.Ns), torch.int32),
            retrieved=((nq, self.Ns), torch.int64), sc=((nq, self.n), torch.uint8),
            hist=((nq, self.Ns + 1), torch.int64), last=((nq,), torch.int32),
            ncand=((nq,), torch.int64), cand=((nq, self.n), torch.int32),
            cand_dist=((nq, self.n), torch.float32), nrecheck=((nq,), torch.int64))
        return {f: torch.empty(shapes[f][0], dtype=shapes[f][1], device=dev) for f in fields}

    def kernel_time(self, kernel: str):
        return tc_kernel_time(self.handle, kernel)

    def profile_reset(self):
        tc_profile_reset(self.handle)

    def batch_capacity(self, beta: float, k_max: int) -> int:
        return tc_batch_capacity(self.handle, beta, k_max)

    def device_errors(self) -> int:
        return tc_device_errors(self.handle)
