"""The larger workloads at their full sizes, in the launch configurations the
benchmark times: invariants on every query, the oracle on a sample.

* 10M x 96 (1M-point k-means training sample, 64 x 64 cells): the FP32 path
  and the benchmark's reduced-precision path (FP8 centroid distances, BF16
  re-rank with the FP32 re-check, autotuned-style launch shapes, one batch,
  graph replay).  With FP8 centroid distances the oracle is fed the GPU's
  distances and must reproduce every later stage.
* 1M x 960: the FP32 path and the BF16 re-rank and centroid distances.
* 1M x 256 with 100,000 queries through tc_search_batched with per-query
  alpha and k (the batched configuration).
"""
import numpy as np
import pytest

import synthdata
from oracle import oracle as O

from gpu_parity import ALL_STAGES, check_topk, compare_query, gpu_search, workload_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def taco_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24919_amd as taco
    taco.load_library()
    return taco


def _setup(name):
    w = synthdata.WORKLOADS[name]
    print(f"[{name}] generating", flush=True)
    X, Q = synthdata.base_and_queries(w)
    print(f"[{name}] index (oracle build if not cached)", flush=True)
    path = workload_index(w, X)
    return w, X, Q, path


def _row_invariants(X, Q, ids, dists, k, n, label):
    """Every row: ids in range and distinct, distances ascending, each the
    squared distance of its id within FP32 summation error, padding last."""
    d = X.shape[1]
    for i in range(ids.shape[0]):
        r, dd = ids[i, :k], dists[i, :k]
        valid = r >= 0
        assert np.all(valid[:valid.sum()]), f"{label} q{i}: padding before results"
        rv = r[valid]
        assert np.all(rv < n) and np.unique(rv).size == rv.size, f"{label} q{i}: ids"
        assert np.all(np.diff(dd[valid]) >= 0) and np.all(np.isinf(dd[~valid])), f"{label} q{i}: order"
        ex = ((X[rv].astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(1)
        assert np.all(np.abs(dd[valid] - ex) <= (d + 4) * 2.0 ** -24 * ex + 1e-30), f"{label} q{i}: dists"


def _downstream_from_gpu_cdist(g, i, qi, oidx, X, Q, alpha, beta, k, label):
    """Alg 4, the counting, Alg 5 and the top-k computed by the oracle's own
    functions on the centroid distances the GPU used (reduced-precision
    forms), compared with every stage the GPU dumped."""
    Ns, n = oidx.Ns, oidx.n
    offs, cid = oidx.offsets(), oidx.ids()
    A, R = O.budget_A(alpha, n), O.budget_R(beta, n)
    sc = np.zeros(n, np.int64)
    for j in range(Ns):
        D1, D2 = g["cdist"][i, j, 0], g["cdist"][i, j, 1]
        i1, i2 = O.argsort(D1), O.argsort(D2)
        assert np.array_equal(g["corder"][i, j, 0], i1) and np.array_equal(g["corder"][i, j, 1], i2), label
        sizes = (offs[j, 1:] - offs[j, :-1]).astype(np.int64)
        cells, got = O.probe(D1, i1, D2, i2, sizes, A)
        assert g["ncells"][i, j] == len(cells) and g["retrieved"][i, j] == got, label
        assert np.array_equal(g["cells"][i, j, :len(cells)], cells), f"{label}: cells j={j}"
        for c in cells:
            sc[cid[j, offs[j, c]:offs[j, c + 1]]] += 1
    assert np.array_equal(g["sc"][i].astype(np.int64), sc), f"{label}: counts"
    hist, last, cand = O.select(sc.astype(np.uint8), Ns, R)
    assert np.array_equal(g["hist"][i], hist) and int(g["last"][i]) == last, f"{label}: threshold"
    nc = int(g["ncand"][i])
    gc = np.sort(g["cand"][i, :nc])
    assert np.array_equal(gc, cand), f"{label}: candidates"
    # top-k of the candidates (ties inside the FP32 tolerance may differ)
    d64 = ((X[cand].astype(np.float64) - Q[qi].astype(np.float64)) ** 2).sum(1)
    top = np.lexsort((cand, d64))[:k]
    oids = np.full(k, -1, np.int64)
    od = np.full(k, np.inf, np.float32)
    oids[:top.size] = cand[top]
    od[:top.size] = d64[top]
    cand_d = np.full(n, np.inf)
    cand_d[cand] = d64
    check_topk(g["ids"][i], g["dists"][i], oids, od, cand_d, label)


def _options(t, torch, w, cd, prec):
    free, _ = torch.cuda.mem_get_info(0)
    return ((t.TC_OPT_CDIST_PRECISION, cd), (t.TC_OPT_PRECISION, prec),
            (t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST), (t.TC_OPT_SCRATCH_BYTES, int(free * 0.6)),
            (t.TC_OPT_MAX_BATCH, w.nq))


def _search_all(t, path, Q, k, alpha, beta, opts, graph=False, calls=1):
    import torch
    idx = t.Index(path, 0)
    try:
        for o, v in opts:
            idx.set_option(o, v)
        if graph:
            idx.set_option(t.TC_OPT_GRAPH, 1)
        q = torch.from_numpy(Q).cuda()
        ids = torch.empty((Q.shape[0], k), dtype=torch.int64, device="cuda")
        dists = torch.empty((Q.shape[0], k), dtype=torch.float32, device="cuda")
        for _ in range(calls):
            ids.fill_(-7)
            idx.search(q, k, alpha, beta, ids=ids, dists=dists)
            torch.cuda.synchronize()
        assert idx.device_errors() == 0
        return ids.cpu().numpy(), dists.cpu().numpy()
    finally:
        idx.close()


def test_sphere_10m_full_size(taco_mod):
    import torch
    t = taco_mod
    w, X, Q, path = _setup("sphere-10m-d96")
    oidx = O.OracleIndex(path)
    alpha, beta, k = 0.005, 0.0003, w.k
    rng = np.random.default_rng(404)
    sample = np.sort(rng.choice(w.nq, 4, replace=False))
    # FP32 path, defaults: every query, then all stages of a sample against the oracle
    print(f"[{w.name}] FP32 path, {w.nq} queries", flush=True)
    idx = t.Index(path, 0)
    g = gpu_search(idx, Q, k, alpha, beta, ("retrieved", "hist", "last", "ncand"))
    A = O.budget_A(alpha, w.n)
    assert np.all(g["hist"].sum(axis=1) == w.n)
    assert np.array_equal((g["hist"] * np.arange(w.Ns + 1)).sum(axis=1), g["retrieved"].sum(axis=1))
    assert np.all(g["retrieved"] >= A)
    _row_invariants(X, Q, g["ids"], g["dists"], k, w.n, "fp32")
    ref = (g["ids"], g["dists"].view(np.uint32))
    print(f"[{w.name}] FP32 path: all stages on {sample.size} queries", flush=True)
    gs = gpu_search(idx, Q[sample], k, alpha, beta, ALL_STAGES)
    idx.close()
    for i, qi in enumerate(sample):
        compare_query(gs, i, oidx.query(Q[qi], alpha, beta, k), w.Ns, k, f"{w.name} q{qi}")
    # the same results from the list form, one batch and graph replays
    print(f"[{w.name}] FP32, list form, one batch, graph", flush=True)
    got = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_FP32, t.TC_FP32),
                      graph=True, calls=2)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1].view(np.uint32), ref[1])
    # FP8 centroid distances: the BF16 re-rank equals the FP32 re-rank on the
    # same probe, bit for bit, for every query; the oracle reproduces every
    # stage from the GPU's distances on the sample
    print(f"[{w.name}] FP8 centroid distances, FP32 and BF16 re-rank", flush=True)
    f32 = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_FP8, t.TC_FP32))
    b16 = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_FP8, t.TC_BF16),
                      graph=True, calls=2)
    assert np.array_equal(b16[0], f32[0]) and np.array_equal(b16[1].view(np.uint32), f32[1].view(np.uint32))
    _row_invariants(X, Q, b16[0], b16[1], k, w.n, "fp8+bf16")
    idx = t.Index(path, 0)
    idx.set_option(t.TC_OPT_CDIST_PRECISION, t.TC_CDIST_FP8)
    gs = gpu_search(idx, Q[sample], k, alpha, beta, ALL_STAGES)
    idx.close()
    for i, qi in enumerate(sample):
        assert np.array_equal(gs["ids"][i], f32[0][qi])
        _downstream_from_gpu_cdist(gs, i, qi, oidx, X, Q, alpha, beta, k, f"{w.name} fp8 q{qi}")
    oidx.close()


def test_aniso_1m_d960_full_size(taco_mod):
    import torch
    t = taco_mod
    w, X, Q, path = _setup("aniso-1m-d960")
    oidx = O.OracleIndex(path)
    alpha, beta, k = 0.1, 0.01, w.k
    rng = np.random.default_rng(960)
    sample = np.sort(rng.choice(w.nq, 6, replace=False))
    print(f"[{w.name}] FP32 path, {w.nq} queries; all stages on {sample.size}", flush=True)
    idx = t.Index(path, 0)
    g = gpu_search(idx, Q, k, alpha, beta, ("retrieved", "hist", "ncand"))
    _row_invariants(X, Q, g["ids"], g["dists"], k, w.n, "fp32")
    gs = gpu_search(idx, Q[sample], k, alpha, beta, ALL_STAGES)
    idx.close()
    for i, qi in enumerate(sample):
        compare_query(gs, i, oidx.query(Q[qi], alpha, beta, k), w.Ns, k, f"{w.name} q{qi}")
    # BF16 re-rank: bit for bit the FP32 results, in the benchmark's launch shapes
    print(f"[{w.name}] BF16 re-rank and BF16 centroid distances", flush=True)
    b16 = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_FP32, t.TC_BF16),
                      graph=True, calls=2)
    assert np.array_equal(b16[0], g["ids"]) and np.array_equal(b16[1].view(np.uint32), g["dists"].view(np.uint32))
    c32 = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_BF16, t.TC_FP32))
    c16 = _search_all(t, path, Q, k, alpha, beta, _options(t, torch, w, t.TC_CDIST_BF16, t.TC_BF16),
                      graph=True, calls=2)
    assert np.array_equal(c16[0], c32[0]) and np.array_equal(c16[1].view(np.uint32), c32[1].view(np.uint32))
    idx = t.Index(path, 0)
    idx.set_option(t.TC_OPT_CDIST_PRECISION, t.TC_CDIST_BF16)
    gs = gpu_search(idx, Q[sample], k, alpha, beta, ALL_STAGES)
    idx.close()
    for i, qi in enumerate(sample):
        _downstream_from_gpu_cdist(gs, i, qi, oidx, X, Q, alpha, beta, k, f"{w.name} bf16 q{qi}")
    oidx.close()


def test_zipf_1m_d256_batched_full_size(taco_mod):
    import torch
    t = taco_mod
    w, X, Q, path = _setup("zipf-1m-d256")
    oidx = O.OracleIndex(path)
    alpha, kq = synthdata.query_budgets(w.nq, w.seed)
    k_max, beta = 100, 0.005
    print(f"[{w.name}] tc_search_batched over {w.nq} queries", flush=True)
    free, _ = torch.cuda.mem_get_info(0)
    idx = t.Index(path, 0)
    idx.set_option(t.TC_OPT_SCRATCH_BYTES, int(free * 0.6))
    idx.set_option(t.TC_OPT_MAX_BATCH, w.nq)
    idx.set_option(t.TC_OPT_GRAPH, 1)
    q = torch.from_numpy(Q).cuda()
    ad, kd = torch.from_numpy(alpha).cuda(), torch.from_numpy(kq).cuda()
    ids = torch.empty((w.nq, k_max), dtype=torch.int64, device="cuda")
    dists = torch.empty((w.nq, k_max), dtype=torch.float32, device="cuda")
    for _ in range(2):
        ids.fill_(-7)
        idx.search_batched(q, ad, kd, k_max, beta, ids=ids, dists=dists)
        torch.cuda.synchronize()
    assert idx.device_errors() == 0
    idx.close()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    for kk in (1, 10, 100):
        rows = np.flatnonzero(kq == kk)
        assert np.all(ids[rows, kk:] == -1) and np.all(np.isinf(dists[rows, kk:])), kk
        _row_invariants(X, Q[rows[:2000]], ids[rows[:2000]], dists[rows[:2000]], kk, w.n, f"k={kk}")
    # the oracle on a sample spanning the three k values and the alpha range
    rng = np.random.default_rng(256)
    sample = np.sort(np.concatenate([rng.choice(np.flatnonzero(kq == kk), 8, replace=False)
                                     for kk in (1, 10, 100)]))
    print(f"[{w.name}] oracle on {sample.size} queries", flush=True)
    for qi in sample:
        r = oidx.query(Q[qi], float(alpha[qi]), beta, int(kq[qi]))
        cand_d = np.full(w.n, np.inf)
        cand_d[r["cand"]] = r["cand_d32"]
        kk = int(kq[qi])
        check_topk(ids[qi, :kk], dists[qi, :kk], r["ids"], r["d32"], cand_d, f"{w.name} q{qi} k={kk}")
    # per-query launches give the same rows
    print(f"[{w.name}] per-query launches on the sample", flush=True)
    idx = t.Index(path, 0)
    for qi in sample:
        kk = int(kq[qi])
        gi, gd = idx.search(q[qi:qi + 1], kk, float(alpha[qi]), beta)
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy()[0], ids[qi, :kk])
        assert np.array_equal(gd.cpu().numpy()[0].view(np.uint32), dists[qi, :kk].view(np.uint32))
    idx.close()
    oidx.close()
