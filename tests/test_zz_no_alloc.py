"""The allocation-free search (tc_search_noalloc) against tc_search.

Its kernels are those of the default split path, with every per-batch buffer
in the library's static device array; results must equal tc_search's with
the default options bit for bit, on consecutive calls that reuse the array
(the second with fewer queries and a smaller k), over several internal
batches, with both Alg 5 readings and the fixed-budget rule.
"""
import numpy as np
import pytest

import synthdata

from gpu_parity import workload_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24919_amd as taco
    # 140k points: a query's scratch is ~1.2 MB, so a call takes a few
    # internal batches of the 256 MiB array
    w = synthdata.WORKLOADS["gmm-int-1m-d128"].scaled("gmm-int-140k-d128", n=140_000, nq=500)
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    print(f"[noalloc] index {path}", flush=True)
    return taco, torch, w, Q, path


def _both(taco, torch, idx, q, k, alpha, beta):
    ids0, d0 = idx.search(q, k, alpha, beta)
    ids1 = torch.full_like(ids0, -7)
    d1 = torch.full_like(d0, -7.0)
    idx.search_noalloc(q, k, alpha, beta, ids1, d1)
    torch.cuda.synchronize()
    return ids0.cpu().numpy(), d0.cpu().numpy(), ids1.cpu().numpy(), d1.cpu().numpy()


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_noalloc_equals_search_on_two_calls(setup, rule):
    taco, torch, w, Q, path = setup
    idx = taco.Index(path, 0)
    try:
        idx.set_option(taco.TC_OPT_SELECT_RULE, rule)
        dev = torch.device("cuda:0")
        for nq, k, alpha, beta in ((500, 10, 0.05, 0.005), (37, 3, 0.02, 0.01)):
            print(f"[noalloc] rule={rule} nq={nq} k={k} alpha={alpha} beta={beta}", flush=True)
            q = torch.from_numpy(np.ascontiguousarray(Q[:nq])).to(dev)
            i0, d0, i1, d1 = _both(taco, torch, idx, q, k, alpha, beta)
            assert np.array_equal(i0, i1), (rule, nq)
            assert np.array_equal(d0.view(np.uint32), d1.view(np.uint32)), (rule, nq)
    finally:
        idx.close()


def test_noalloc_ignores_other_forms_and_rejects_bad_arguments(setup):
    # the index's options select the list form, the 8-bit re-rank and FP8
    # centroid distances; the allocation-free call keeps the plain FP32 path
    taco, torch, w, Q, path = setup
    dev = torch.device("cuda:0")
    q = torch.from_numpy(np.ascontiguousarray(Q[:64])).to(dev)
    ref = taco.Index(path, 0)
    i0, d0 = ref.search(q, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    ref.close()
    idx = taco.Index(path, 0)
    try:
        idx.set_option(taco.TC_OPT_COUNT_MODE, taco.TC_COUNT_LIST)
        idx.set_option(taco.TC_OPT_PRECISION, taco.TC_U8)
        idx.set_option(taco.TC_OPT_CDIST_PRECISION, taco.TC_CDIST_FP8)
        ids = torch.empty((64, 10), dtype=torch.int64, device=dev)
        dists = torch.empty((64, 10), dtype=torch.float32, device=dev)
        idx.search_noalloc(q, 10, 0.05, 0.005, ids, dists)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), i0.cpu().numpy())
        assert np.array_equal(dists.cpu().numpy().view(np.uint32), d0.cpu().numpy().view(np.uint32))
        L = taco.load_library()
        for args in ((q.data_ptr(), 64, 0, 0.05, 0.005), (q.data_ptr(), 64, 10, 0.0, 0.005),
                     (q.data_ptr(), 64, 10, 0.05, 1.5), (None, 64, 10, 0.05, 0.005)):
            rc = L.tc_search_noalloc(idx.handle, *args, ids.data_ptr(), dists.data_ptr(), None)
            assert rc == taco.TC_EINVAL, args
    finally:
        idx.close()
