"""Bounded candidate slots (TC_OPT_CANDIDATE_SLOTS) on the GPU.

Alg 5 (Section 4.3) keeps the whole threshold level, so a query's candidate
set |C| = S(last) is about R = floor(beta*n) but can reach n.  A call gives
each query max(S, 8R, 32*k_max) slots (S = TC_OPT_CANDIDATE_SLOTS); a query
with more candidates skips the slots and takes the streamed FP32 re-rank and
top-k over its packed counts.  Its results must be bit-identical to the full-slot
path (cap = n, which the oracle parity tests cover) in every count form,
under both threshold readings, for the reduced-precision re-ranks (which
re-check in FP32), and in the batched and allocation-free entry points.
The list form's per-tile lists (W*bits/32 slots per tile) overflow into the
recount the same way.  Whether a query overflows is read from the stage
dumps (they always hold every candidate), so each test also shows that its
settings make some queries take the streamed path.
"""
import numpy as np
import pytest

import synthdata

from gpu_parity import workload_index

pytestmark = pytest.mark.gpu

SMALL = 16  # candidate slots per query planned for: overflow is common


@pytest.fixture(scope="module")
def taco_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24919_amd as taco
    taco.load_library()
    return taco


@pytest.fixture(scope="module")
def tiny(taco_mod):
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"]
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    return dict(w=w, X=X, Q=Q, path=path)


def _search(taco, path, Q, k, alpha, beta, options=(), launches=None):
    """Results of one call; with `launches` (a list), appends the number of
    streamed top-k launches the call made."""
    import torch
    idx = taco.Index(path, 0)
    try:
        for opt, val in options:
            idx.set_option(opt, val)
        if launches is not None:
            idx.set_option(taco.TC_OPT_PROFILE, 1)
        ids, dists = idx.search(torch.from_numpy(Q).cuda(), k, alpha, beta)
        torch.cuda.synchronize()
        assert idx.device_errors() == 0
        if launches is not None:
            launches.append(idx.kernel_time("stream")[1])
        return ids.cpu().numpy(), dists.cpu().numpy()
    finally:
        idx.close()


def _ncand(taco, path, Q, k, alpha, beta, rule):
    """|C| per query, from the stage dumps."""
    import torch
    idx = taco.Index(path, 0)
    try:
        idx.set_option(taco.TC_OPT_SELECT_RULE, rule)
        dump = idx.dump_buffers(Q.shape[0], ("ncand",))
        idx.search_debug(torch.from_numpy(Q).cuda(), k, alpha, beta, dump)
        torch.cuda.synchronize()
        return dump["ncand"].cpu().numpy()
    finally:
        idx.close()


def _cap(n, beta, slots, k_max=10):
    R = int(np.floor(beta * n))
    return min(n, max(slots, 8 * R, 32 * k_max))


def _same(a, b, label):
    assert np.array_equal(a[0], b[0]), f"{label}: ids differ"
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32)), f"{label}: distance bits differ"


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("alpha,beta", [(0.2, 0.001), (0.3, 0.0005), (0.003, 0.005)])
def test_streamed_topk_equals_full_slots(taco_mod, tiny, rule, alpha, beta):
    t = taco_mod
    Q, path, n = tiny["Q"], tiny["path"], tiny["w"].n
    nc = _ncand(t, path, Q, 10, alpha, beta, rule)
    over = int(np.sum(nc > _cap(n, beta, SMALL)))
    print(f"[slots] a={alpha} b={beta} rule={rule}: {over}/{len(nc)} queries overflow "
          f"cap {_cap(n, beta, SMALL)} (|C| max {nc.max()})", flush=True)
    assert over > 0, "these settings should overflow some queries"
    modes = (t.TC_COUNT_SPLIT, t.TC_COUNT_FUSED, t.TC_COUNT_LIST, t.TC_COUNT_CODES)
    for mode in modes:
        base = ((t.TC_OPT_SELECT_RULE, rule), (t.TC_OPT_COUNT_MODE, mode), (t.TC_OPT_TILE_IDS, 4096))
        full = _search(t, path, Q, 10, alpha, beta, base + ((t.TC_OPT_CANDIDATE_SLOTS, n),))
        small = _search(t, path, Q, 10, alpha, beta, base + ((t.TC_OPT_CANDIDATE_SLOTS, SMALL),))
        _same(full, small, f"mode {mode}")
    for prec in (t.TC_BF16, t.TC_U8):
        base = ((t.TC_OPT_SELECT_RULE, rule), (t.TC_OPT_PRECISION, prec))
        ref = _search(t, path, Q, 10, alpha, beta, ((t.TC_OPT_SELECT_RULE, rule),
                                                    (t.TC_OPT_CANDIDATE_SLOTS, n)))
        small = _search(t, path, Q, 10, alpha, beta, base + ((t.TC_OPT_CANDIDATE_SLOTS, SMALL),))
        # the bounded re-ranks re-check every row that can reach the top k in
        # FP32: their results are the FP32 path's
        _same(ref, small, f"precision {prec}")


def test_fixed_rule_never_streams(taco_mod, tiny):
    """The fixed-budget rule selects exactly min(R, ...) <= cap candidates."""
    t = taco_mod
    Q, path, n = tiny["Q"], tiny["path"], tiny["w"].n
    opts = ((t.TC_OPT_SELECT_RULE, t.TC_RULE_FIXED),)
    full = _search(t, path, Q, 10, 0.2, 0.001, opts + ((t.TC_OPT_CANDIDATE_SLOTS, n),))
    launches = []
    small = _search(t, path, Q, 10, 0.2, 0.001, opts + ((t.TC_OPT_CANDIDATE_SLOTS, SMALL),), launches)
    _same(full, small, "fixed rule")
    assert launches == [0]
    # the same slots with the printed reading do stream
    _search(t, path, Q, 10, 0.2, 0.001, ((t.TC_OPT_CANDIDATE_SLOTS, SMALL),), launches)
    assert launches[1] >= 1


@pytest.mark.parametrize("level", [1, 0])
def test_list_tile_overflow_takes_the_recount(taco_mod, tiny, level):
    """1024-id tiles hold 128 list slots each (4-bit counts): at alpha = 0.2
    and list level 1 most tiles list more, so those queries are counted
    again; the results are the split form's."""
    import torch
    t = taco_mod
    Q, path, n = tiny["Q"], tiny["path"], tiny["w"].n
    idx = t.Index(path, 0)
    try:
        idx.set_option(t.TC_OPT_TILE_IDS, 1024)
        dump = idx.dump_buffers(Q.shape[0], ("sc",))
        idx.search_debug(torch.from_numpy(Q).cuda(), 10, 0.2, 0.001, dump)
        torch.cuda.synchronize()
        sc = dump["sc"].cpu().numpy()
    finally:
        idx.close()
    pad = (-n) % 1024
    per_tile = (np.pad(sc, ((0, 0), (0, pad))) >= 1).reshape(sc.shape[0], -1, 1024).sum(axis=2)
    print(f"[slots] list level {level}: tiles listing > 128 ids at level 1: "
          f"{int(np.sum(per_tile > 128))} of {per_tile.size}", flush=True)
    assert np.any(per_tile > 128)
    split = _search(t, path, Q, 10, 0.2, 0.001, ((t.TC_OPT_TILE_IDS, 1024),
                                                 (t.TC_OPT_COUNT_MODE, t.TC_COUNT_SPLIT)))
    for slots in (n, SMALL):
        lst = _search(t, path, Q, 10, 0.2, 0.001, (
            (t.TC_OPT_TILE_IDS, 1024), (t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST),
            (t.TC_OPT_LIST_LEVEL, level), (t.TC_OPT_CANDIDATE_SLOTS, slots), (t.TC_OPT_MAX_BATCH, 13)))
        _same(split, lst, f"list level {level} slots {slots}")


def test_batched_and_noalloc_stream(taco_mod, tiny):
    import torch
    t = taco_mod
    Q, path, n = tiny["Q"], tiny["path"], tiny["w"].n
    nq = Q.shape[0]
    nc = _ncand(t, path, Q, 10, 0.003, 0.005, 0)
    assert np.any(nc > _cap(n, 0.005, SMALL)), "these settings should overflow some queries"
    rng = np.random.default_rng(5)
    alpha = np.exp(rng.uniform(np.log(0.003), np.log(0.05), nq))
    kk = rng.choice(np.array([1, 10], dtype=np.int32), nq).astype(np.int32)
    q = torch.from_numpy(Q).cuda()
    out = {}
    for slots in (n, SMALL):
        idx = t.Index(path, 0)
        try:
            idx.set_option(t.TC_OPT_CANDIDATE_SLOTS, slots)
            ids, d = idx.search_batched(q, torch.from_numpy(alpha).cuda(), torch.from_numpy(kk).cuda(),
                                        10, 0.005)
            nids = torch.empty((nq, 10), dtype=torch.int64, device="cuda")
            nd = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
            idx.search_noalloc(q, 10, 0.003, 0.005, nids, nd)
            torch.cuda.synchronize()
            assert idx.device_errors() == 0
            out[slots] = (ids.cpu().numpy(), d.cpu().numpy(), nids.cpu().numpy(), nd.cpu().numpy())
        finally:
            idx.close()
    a, b = out[n], out[SMALL]
    _same(a[:2], b[:2], "batched")
    _same(a[2:], b[2:], "noalloc")
    ref = _search(t, path, Q, 10, 0.003, 0.005, ((t.TC_OPT_CANDIDATE_SLOTS, n),))
    _same(ref, a[2:], "noalloc vs search")


def test_batch_capacity_follows_beta(taco_mod, tiny):
    t = taco_mod
    path, n = tiny["path"], tiny["w"].n
    idx = t.Index(path, 0)
    try:
        idx.set_option(t.TC_OPT_CANDIDATE_SLOTS, SMALL)
        idx.set_option(t.TC_OPT_MAX_BATCH, 7)
        # pool = max(7 * 16, n) = n slots
        assert idx.batch_capacity(0.02, 10) == min(7, n // _cap(n, 0.02, SMALL))
        assert idx.batch_capacity(0.2, 10) == n // _cap(n, 0.2, SMALL) == 1
        assert idx.batch_capacity(0.5, 10) == 1  # cap = n
        assert idx.batch_capacity(0.0, 10) == 7
        with pytest.raises(Exception):
            idx.batch_capacity(1.5, 10)
        with pytest.raises(Exception):
            idx.batch_capacity(0.1, 0)
    finally:
        idx.close()


def test_one_query_per_batch_at_large_beta(taco_mod, tiny):
    """beta = 0.5: every query takes all n slots, one per batch."""
    t = taco_mod
    Q, path, n = tiny["Q"], tiny["path"], tiny["w"].n
    ref = _search(t, path, Q[:9], 10, 0.05, 0.5)
    one = _search(t, path, Q[:9], 10, 0.05, 0.5, ((t.TC_OPT_CANDIDATE_SLOTS, SMALL),
                                                  (t.TC_OPT_MAX_BATCH, 4)))
    _same(ref, one, "beta 0.5")
