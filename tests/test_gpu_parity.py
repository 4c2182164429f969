"""GPU path vs the CPU oracle, through the C-ABI.

Bit-exact: transformed queries, half-centroid distances, their order, probed
cells, retrieved counts, collision counts, level histograms, thresholds and
candidate sets.  Within 1e-5 relative: re-rank distances.  Result ids equal
except at distance ties inside that tolerance.
"""
import numpy as np
import pytest

import synthdata
from oracle import oracle as O

from gpu_parity import ALL_STAGES, compare_query, gpu_search, scaled_workloads, workload_index

pytestmark = pytest.mark.gpu


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
    print(f"[tiny] index {path}", flush=True)
    return dict(w=w, X=X, Q=Q, path=path, oidx=O.OracleIndex(path))


def _run_all(taco, path, oidx, Q, k, alpha, beta, rule, label, options=()):
    idx = taco.Index(path, 0)
    try:
        idx.set_option(taco.TC_OPT_SELECT_RULE, rule)
        for opt, val in options:
            idx.set_option(opt, val)
        g = gpu_search(idx, Q, k, alpha, beta, ALL_STAGES)
    finally:
        idx.close()
    for qi in range(Q.shape[0]):
        r = oidx.query(Q[qi], alpha, beta, k, rule=rule)
        compare_query(g, qi, r, oidx.Ns, k, label)
    return g


@pytest.mark.parametrize("alpha,beta,rule", [
    (0.05, 0.005, 0), (0.05, 0.005, 1), (0.01, 0.02, 0), (0.2, 0.001, 0), (0.003, 0.05, 1)])
def test_tiny_all_stages(taco_mod, tiny, alpha, beta, rule):
    print(f"[tiny] alpha={alpha} beta={beta} rule={rule}", flush=True)
    _run_all(taco_mod, tiny["path"], tiny["oidx"], tiny["Q"], 10, alpha, beta, rule,
             f"tiny a={alpha} b={beta} r={rule}")


def test_tiny_multi_tile_and_multi_batch(taco_mod, tiny):
    # 4096-id tiles: 20000 ids = 4 full tiles + a ragged tail of 3616; batches
    # of 7 queries: 14 full batches + a ragged batch of 2.
    print("[tiny] tile=4096 batch=7", flush=True)
    t = taco_mod
    _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 0, "tiny tiles",
             options=((t.TC_OPT_TILE_IDS, 4096), (t.TC_OPT_MAX_BATCH, 7)))


def test_tiny_alpha_beta_one_is_exact_knn(taco_mod, tiny):
    print("[tiny] alpha=beta=1", flush=True)
    idx = taco_mod.Index(tiny["path"], 0)
    g = gpu_search(idx, tiny["Q"][:16], 25, 1.0, 1.0, ("sc", "ncand", "last"))
    idx.close()
    gi, gd = O.bruteforce(tiny["X"], tiny["Q"][:16], 25)
    assert np.all(g["sc"] == 8) and np.all(g["ncand"] == tiny["w"].n)
    assert np.array_equal(g["ids"], gi)
    np.testing.assert_allclose(g["dists"], gd, rtol=1e-5)


def test_tiny_k_edges_and_padding(taco_mod, tiny):
    print("[tiny] k edges", flush=True)
    Q, oidx = tiny["Q"][:6], tiny["oidx"]
    for k, alpha, beta in ((1, 0.05, 0.005), (1024, 0.0001, 0.0), (100, 0.02, 0.002)):
        idx = taco_mod.Index(tiny["path"], 0)
        g = gpu_search(idx, Q, k, alpha, beta, ALL_STAGES)
        idx.close()
        for qi in range(Q.shape[0]):
            compare_query(g, qi, oidx.query(Q[qi], alpha, beta, k), oidx.Ns, k, f"k={k}")


def test_empty_batch_and_argument_errors(taco_mod, tiny):
    import torch
    t = taco_mod
    idx = t.Index(tiny["path"], 0)
    q0 = torch.empty((0, tiny["w"].d), dtype=torch.float32, device="cuda:0")
    ids, dists = idx.search(q0, 10, 0.05, 0.005)
    assert ids.shape == (0, 10)
    q = torch.from_numpy(tiny["Q"][:2]).cuda()
    for k, a, b in ((0, 0.05, 0.005), (1025, 0.05, 0.005), (10, 0.0, 0.005), (10, 1.5, 0.005),
                    (10, 0.05, -0.1), (10, 0.05, 1.01), (tiny["w"].n + 1, 0.05, 0.005)):
        with pytest.raises(t.TacoError) as e:
            idx.search(q, k, a, b)
        assert e.value.code == t.TC_EINVAL
    with pytest.raises(t.TacoError):
        idx.set_option(t.TC_OPT_TILE_IDS, 1000)
    idx.close()


def test_deterministic_across_tiles_and_batches(taco_mod, tiny):
    t = taco_mod
    outs = []
    for tile, batch in ((65536, 4096), (8192, 33), (2048, 1)):
        idx = t.Index(tiny["path"], 0)
        idx.set_option(t.TC_OPT_TILE_IDS, tile)
        idx.set_option(t.TC_OPT_MAX_BATCH, batch)
        outs.append(gpu_search(idx, tiny["Q"][:40], 10, 0.05, 0.005, ("sc", "hist", "ncand")))
        idx.close()
    for o in outs[1:]:
        for f in ("sc", "hist", "ncand", "ids"):
            assert np.array_equal(o[f], outs[0][f]), f
        assert np.array_equal(o["dists"].view(np.uint32), outs[0]["dists"].view(np.uint32))


@pytest.mark.parametrize("w", scaled_workloads(), ids=lambda w: w.name)
def test_workload_shapes_all_stages(taco_mod, w):
    X, Q = synthdata.base_and_queries(w)
    print(f"[{w.name}] building index", flush=True)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    t = taco_mod
    for alpha, beta, rule, opts in ((0.05, 0.005, 0, ()), (0.02, 0.01, 1, ((t.TC_OPT_TILE_IDS, 8192),))):
        print(f"[{w.name}] alpha={alpha} beta={beta} rule={rule}", flush=True)
        _run_all(t, path, oidx, Q, 10, alpha, beta, rule, w.name, options=opts)


def test_bench_workload_full_size_sampled(taco_mod):
    """The 1M x 128 workload at its full size, in the launch configuration
    the benchmark times (default options, all 10,000 queries in one call):
    invariants on every query, the oracle on a sample of queries."""
    w = synthdata.WORKLOADS["gmm-int-1m-d128"]
    print(f"[{w.name}] generating", flush=True)
    X, Q = synthdata.base_and_queries(w)
    print(f"[{w.name}] index (oracle build if not cached)", flush=True)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    idx = taco_mod.Index(path, 0)
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(w.nq, 12, replace=False))
    small = ("retrieved", "ncells", "hist", "last", "ncand")
    ref = {}
    for alpha in w.alphas:
        print(f"[{w.name}] alpha={alpha}: full batch", flush=True)
        g = gpu_search(idx, Q, w.k, alpha, w.beta, small)
        ref[alpha] = (g["ids"], g["dists"].view(np.uint32))
        A = O.budget_A(alpha, w.n)
        levels = np.arange(w.Ns + 1)
        assert np.all(g["hist"].sum(axis=1) == w.n)
        assert np.array_equal((g["hist"] * levels).sum(axis=1), g["retrieved"].sum(axis=1))
        assert np.all(g["retrieved"] >= A)
        lastc = np.maximum(g["last"], 0)
        want_nc = np.array([g["hist"][i, lastc[i]:].sum() for i in range(w.nq)])
        assert np.array_equal(g["ncand"], want_nc)
        assert np.all(g["dists"][:, 1:] >= g["dists"][:, :-1])
        for qi in sample:
            r = oidx.query(Q[qi], alpha, w.beta, w.k)
            compare_query(g, qi, r, w.Ns, w.k, f"{w.name} a={alpha}")
        print(f"[{w.name}] alpha={alpha}: all stages on the sample", flush=True)
        gs = gpu_search(idx, Q[sample[:4]], w.k, alpha, w.beta, ALL_STAGES)
        for i, qi in enumerate(sample[:4]):
            compare_query(gs, i, oidx.query(Q[qi], alpha, w.beta, w.k), w.Ns, w.k, f"{w.name} a={alpha}")
    idx.close()
    # the benchmark's tuned configuration: list selection, exact 8-bit re-rank,
    # 8 re-rank and 2 probe queries per workgroup, all 10,000 queries in one
    # batch, replayed from a graph; bit for bit the results above
    import torch
    t = taco_mod
    free, _ = torch.cuda.mem_get_info(0)
    opts = ((t.TC_OPT_PRECISION, t.TC_U8), (t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST),
            (t.TC_OPT_RERANK_BLOCKS, 8), (t.TC_OPT_PROBE_QPW, 2),
            (t.TC_OPT_SCRATCH_BYTES, int(free * 0.6)), (t.TC_OPT_MAX_BATCH, w.nq))
    for alpha in w.alphas:
        print(f"[{w.name}] alpha={alpha}: tuned configuration", flush=True)
        got = _search_bits(t, path, Q, alpha, opts, calls=2, graph=True)
        assert np.array_equal(got[0], ref[alpha][0]) and np.array_equal(got[1], ref[alpha][1]), alpha


def _bf16_cases():
    W = synthdata.WORKLOADS
    return [W["tiny-gmm-20k-d128"]] + scaled_workloads()


@pytest.mark.parametrize("prec", ["bf16", "u8"])
@pytest.mark.parametrize("w", _bf16_cases(), ids=lambda w: w.name)
def test_bounded_rerank_equals_fp32(taco_mod, w, prec):
    """The BF16 and 8-bit re-ranks with their FP32 boundary re-check return
    exactly the FP32 path's ids and distances (bit for bit), re-checking a
    subset of the candidates."""
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    print(f"[{w.name}] {prec} vs fp32", flush=True)
    for k, alpha, beta in ((10, 0.05, 0.005), (1, 0.02, 0.01), (100, 0.01, 0.02)):
        idx = t.Index(path, 0)
        g32 = gpu_search(idx, Q, k, alpha, beta, ("ncand",))
        idx.set_option(t.TC_OPT_PRECISION, t.TC_BF16 if prec == "bf16" else t.TC_U8)
        g16 = gpu_search(idx, Q, k, alpha, beta, ("ncand", "nrecheck"))
        idx.close()
        assert np.array_equal(g16["ids"], g32["ids"]), (w.name, k)
        assert np.array_equal(g16["dists"].view(np.uint32), g32["dists"].view(np.uint32)), (w.name, k)
        nr, nc = g16["nrecheck"], g16["ncand"]
        # 0 where the 8-bit bounds are the distances (integer queries on
        # integer rows); otherwise at least the k kept rows
        assert np.all((nr >= np.minimum(k, nc)) | ((nr == 0) & (prec == "u8"))) and np.all(nr <= nc)
        print(f"[{w.name}] k={k}: re-checked {nr.mean():.1f} of {nc.mean():.0f} candidates", flush=True)


def test_u8_integer_queries_and_others_equal_fp32(taco_mod):
    """On integer rows in [0, 255] the 8-bit re-rank takes exact byte dot
    products for queries of integers in [0, 255] and the bounded form for the
    rest; a batch mixing both (queries shifted by fractions, negative or
    above 255 in one coordinate) matches the FP32 path bit for bit, also in
    ragged batches, and the exact form re-checks no row."""
    t = taco_mod
    w = synthdata.WORKLOADS["gmm-int-1m-d128"].scaled("gmm-int-40k-d128-q48", n=40_000, nq=48)
    X, Q = synthdata.base_and_queries(w)
    assert np.all(X == np.round(X)) and X.min() >= 0 and X.max() <= 255
    path = workload_index(w, X)
    Q = Q.copy()
    n_int = Q.shape[0] // 2
    Q[n_int::3] += 0.25
    Q[n_int + 1::3, 5] = -1.0
    Q[n_int + 2::3, 7] = 256.0
    for k, alpha, beta, mb in ((10, 0.05, 0.005, 0), (100, 0.01, 0.02, 0), (10, 0.05, 0.005, 13)):
        # mb: batches of 13 (a ragged last one)
        idx = t.Index(path, 0)
        g32 = gpu_search(idx, Q, k, alpha, beta, ("ncand",))
        idx.set_option(t.TC_OPT_PRECISION, t.TC_U8)
        if mb:
            idx.set_option(t.TC_OPT_MAX_BATCH, mb)
        g8 = gpu_search(idx, Q, k, alpha, beta, ("ncand", "nrecheck"))
        idx.close()
        assert np.array_equal(g8["ids"], g32["ids"]), k
        assert np.array_equal(g8["dists"].view(np.uint32), g32["dists"].view(np.uint32)), k
        nr = g8["nrecheck"]
        # both bounds are the distance: the top k of the bounds is the
        # result, and no row is re-checked
        assert np.all(nr[:n_int] == 0), nr[:n_int]
        assert np.all(nr[n_int:] >= np.minimum(k, g8["ncand"][n_int:]))
        print(f"[{w.name}] u8 integer queries k={k}: re-checked {nr[:n_int].mean():.1f}; "
              f"others {nr[n_int:].mean():.1f} of {g8['ncand'][n_int:].mean():.0f}", flush=True)


@pytest.mark.parametrize("mode", ["split", "fused", "list", "codes"])
def test_count_modes_all_stages(taco_mod, tiny, mode):
    """The split (count, then select), fused (one cooperative launch), list
    (ids at or above the list level listed while counting) and point-major
    (cell codes against probed-cell bitmaps) paths all match the oracle
    stage by stage, also with several tiles per query and several batches."""
    t = taco_mod
    m = {"split": t.TC_COUNT_SPLIT, "fused": t.TC_COUNT_FUSED, "list": t.TC_COUNT_LIST,
         "codes": t.TC_COUNT_CODES}[mode]
    print(f"[tiny] count mode {mode}", flush=True)
    for opts in (((t.TC_OPT_COUNT_MODE, m),),
                 ((t.TC_OPT_TILE_IDS, 4096), (t.TC_OPT_COUNT_MODE, m), (t.TC_OPT_MAX_BATCH, 13))):
        _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 0, f"tiny {mode}",
                 options=opts)


@pytest.mark.parametrize("cqpw", [2, 4, 32])
@pytest.mark.parametrize("mode", ["split", "list"])
def test_count_queries_per_workgroup_all_stages(taco_mod, tiny, mode, cqpw):
    """Counting workgroups that take several queries of their tile in turn
    (the last one partly empty) match the oracle stage by stage."""
    t = taco_mod
    m = {"split": t.TC_COUNT_SPLIT, "list": t.TC_COUNT_LIST}[mode]
    print(f"[tiny] count mode {mode}, {cqpw} queries per workgroup", flush=True)
    for opts in (((t.TC_OPT_COUNT_MODE, m), (t.TC_OPT_COUNT_QPW, cqpw)),
                 ((t.TC_OPT_TILE_IDS, 4096), (t.TC_OPT_COUNT_MODE, m), (t.TC_OPT_COUNT_QPW, cqpw),
                  (t.TC_OPT_MAX_BATCH, 13))):
        _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 0, f"tiny {mode} cqpw={cqpw}",
                 options=opts)


@pytest.mark.parametrize("mode", ["split", "list"])
def test_count_workgroup_768_all_stages(taco_mod, tiny, mode):
    """768-thread counting workgroups (TC_OPT_COUNT_BLOCK) match the oracle
    stage by stage: whole tiles and 4096-id tiles with a ragged tail, one and
    several queries per workgroup, batches with a ragged end."""
    t = taco_mod
    m = {"split": t.TC_COUNT_SPLIT, "list": t.TC_COUNT_LIST}[mode]
    print(f"[tiny] count mode {mode}, 768-thread workgroups", flush=True)
    for opts in (((t.TC_OPT_COUNT_MODE, m), (t.TC_OPT_COUNT_BLOCK, 768)),
                 ((t.TC_OPT_TILE_IDS, 4096), (t.TC_OPT_COUNT_MODE, m), (t.TC_OPT_COUNT_BLOCK, 768),
                  (t.TC_OPT_COUNT_QPW, 4), (t.TC_OPT_MAX_BATCH, 13))):
        _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 0, f"tiny {mode} nt=768",
                 options=opts)


def test_count_workgroup_sizes_same_results(taco_mod, tiny):
    """Without stage dumps (the re-walk listing, the multi-query forms), both
    workgroup sizes give bit-identical results in every split and list
    configuration, at list levels the re-walk and the scan both serve."""
    import torch
    t = taco_mod
    q = torch.from_numpy(tiny["Q"]).cuda()

    def run(opts):
        idx = t.Index(tiny["path"], 0)
        try:
            for opt, val in opts:
                idx.set_option(opt, val)
            ids, d = idx.search(q, 10, 0.05, 0.005)
            torch.cuda.synchronize()
            assert idx.device_errors() == 0
            return ids.cpu().numpy(), d.cpu().numpy().view(np.uint32)
        finally:
            idx.close()

    for mode in (t.TC_COUNT_SPLIT, t.TC_COUNT_LIST):
        for tile in (131072, 4096):
            for cqpw in (1, 8):
                for level in (0, 1, 3):
                    base = ((t.TC_OPT_COUNT_MODE, mode), (t.TC_OPT_TILE_IDS, tile),
                            (t.TC_OPT_COUNT_QPW, cqpw), (t.TC_OPT_LIST_LEVEL, level))
                    a = run(base + ((t.TC_OPT_COUNT_BLOCK, 1024),))
                    b = run(base + ((t.TC_OPT_COUNT_BLOCK, 768),))
                    lab = f"mode {mode} tile {tile} cqpw {cqpw} level {level}"
                    assert np.array_equal(a[0], b[0]), f"{lab}: ids differ"
                    assert np.array_equal(a[1], b[1]), f"{lab}: distance bits differ"
    with pytest.raises(Exception):
        run(((t.TC_OPT_COUNT_BLOCK, 512),))


@pytest.mark.parametrize("qpw", [1, 2, 8, 16])
def test_probe_widths_all_stages(taco_mod, tiny, qpw):
    """Every probe workgroup width (queries per workgroup) matches the oracle
    stage by stage, also when the batch leaves the last workgroup partly
    empty."""
    t = taco_mod
    print(f"[tiny] probe queries per workgroup {qpw}", flush=True)
    for opts in (((t.TC_OPT_PROBE_QPW, qpw),), ((t.TC_OPT_PROBE_QPW, qpw), (t.TC_OPT_MAX_BATCH, 13))):
        _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 0, f"tiny qpw {qpw}",
                 options=opts)


@pytest.mark.parametrize("level", [1, 2, 3, 4, 8])
def test_list_levels_all_stages(taco_mod, tiny, level):
    """Every fixed list level matches the oracle stage by stage: queries whose
    threshold is below the level (recounted and selected from their packed
    counts), at it (the list is the candidate set) and above it (the list is
    filtered)."""
    t = taco_mod
    print(f"[tiny] list level {level}", flush=True)
    seen = np.zeros(3, np.int64)
    for alpha, beta in ((0.05, 0.005), (0.01, 0.02), (0.2, 0.001)):
        for opts in (((t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST), (t.TC_OPT_LIST_LEVEL, level)),
                     ((t.TC_OPT_TILE_IDS, 4096), (t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST),
                      (t.TC_OPT_LIST_LEVEL, level), (t.TC_OPT_MAX_BATCH, 13))):
            g = _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, alpha, beta, 0,
                         f"tiny list level {level} a={alpha}", options=opts)
            last = g["last"].astype(np.int64)
            seen += [(last < level).sum(), (last == level).sum(), (last > level).sum()]
    print(f"[tiny] list level {level}: below/at/above {seen.tolist()}", flush=True)


def _search_bits(t, path, Q, alpha, options, calls=1, graph=False):
    """Results of `calls` searches (no dumps) with the given options; all
    calls must agree bit for bit."""
    import torch
    idx = t.Index(path, 0)
    try:
        for opt, val in options:
            idx.set_option(opt, val)
        if graph:
            idx.set_option(t.TC_OPT_GRAPH, 1)
        q = torch.from_numpy(Q).cuda()
        out = None
        for c in range(calls):
            ids, d = idx.search(q, 10, alpha, 0.005)
            torch.cuda.synchronize()
            r = (ids.cpu().numpy(), d.cpu().numpy().view(np.uint32))
            if out is None:
                out = r
            else:
                assert np.array_equal(out[0], r[0]) and np.array_equal(out[1], r[1]), c
            _ = (q * 2.0).sum().item()  # eager work between calls
        assert idx.device_errors() == 0
    finally:
        idx.close()
    return out


@pytest.mark.parametrize("w", [synthdata.WORKLOADS["tiny-gmm-20k-d128"]] + scaled_workloads(),
                         ids=lambda w: w.name)
def test_list_mode_equals_split_without_dumps(taco_mod, w):
    """Without stage dumps (the product path: no packed counts stored unless
    queued), the list path gives the split path's results bit for bit, at the
    adaptive level across repeated calls and batches (the level moves on the
    device between them), at fixed levels, and replayed from a graph."""
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    Ns = w.Ns
    print(f"[{w.name}] list vs split, no dumps", flush=True)
    for alpha in (0.01, 0.05, 0.2):
        ref = _search_bits(t, path, Q, alpha, ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_SPLIT),))
        for level in sorted({0, 1, 3, Ns}):
            for mb in (0, 7):
                opts = [(t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST), (t.TC_OPT_LIST_LEVEL, level)]
                if mb:
                    opts.append((t.TC_OPT_MAX_BATCH, mb))
                got = _search_bits(t, path, Q, alpha, opts, calls=3)
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (alpha, level, mb)
        got = _search_bits(t, path, Q, alpha, ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST),
                                               (t.TC_OPT_MAX_BATCH, 5)), calls=4, graph=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (alpha, "graph")


def test_list_mode_many_tiles(taco_mod):
    """Past the tiles the list selection groups (137 tiles of 1,024 ids), its
    candidates stay ungrouped and the re-rank takes them interleaved; with 18
    tiles they are grouped by tile and the exact 8-bit re-rank hands each tile
    residue to its own workgroups.  Both equal the split path bit for bit, in
    FP32 and in the 8-bit re-rank, with 8 and 16 re-rank workgroups."""
    t = taco_mod
    w = synthdata.WORKLOADS["gmm-int-1m-d128"].scaled("gmm-int-140k-d128", n=140_000, nq=16)
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    print(f"[{w.name}] list vs split, many tiles", flush=True)
    for prec in (t.TC_FP32, t.TC_U8):
        for tile in (1024, 8192):
            base = ((t.TC_OPT_PRECISION, prec), (t.TC_OPT_TILE_IDS, tile))
            ref = _search_bits(t, path, Q, 0.05, base + ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_SPLIT),))
            for rr in (8, 16):
                got = _search_bits(t, path, Q, 0.05, base + ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST),
                                                             (t.TC_OPT_RERANK_BLOCKS, rr)), calls=2)
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (prec, tile, rr)


@pytest.mark.parametrize("w", scaled_workloads(), ids=lambda w: w.name)
def test_workload_shapes_split_mode(taco_mod, w):
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    print(f"[{w.name}] split mode", flush=True)
    _run_all(t, path, oidx, Q, 10, 0.05, 0.005, 0, w.name + " split",
             options=((t.TC_OPT_COUNT_MODE, t.TC_COUNT_SPLIT),))


def _batched_inputs(w, nq, seed=5):
    alpha, k = synthdata.query_budgets(nq, seed)
    return alpha, k


@pytest.mark.parametrize("w", [synthdata.WORKLOADS["tiny-gmm-20k-d128"]] + scaled_workloads()[3:],
                         ids=lambda w: w.name)
def test_batched_per_query_budgets(taco_mod, w):
    """tc_search_batched with query-aware budgets (alpha log-uniform in
    [0.005, 0.1], k in {1, 10, 100}) matches the oracle query by query."""
    import torch
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    alpha, k = _batched_inputs(w, Q.shape[0])
    k_max = 100
    print(f"[{w.name}] batched budgets", flush=True)
    for prec in (t.TC_FP32, t.TC_BF16):
        idx = t.Index(path, 0)
        idx.set_option(t.TC_OPT_PRECISION, prec)
        q = torch.from_numpy(Q).cuda()
        ids, dists = idx.search_batched(q, torch.from_numpy(alpha).cuda(), torch.from_numpy(k).cuda(),
                                        k_max, 0.005)
        torch.cuda.synchronize()
        assert idx.device_errors() == 0
        ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
        idx.close()
        for qi in range(Q.shape[0]):
            r = oidx.query(Q[qi], float(alpha[qi]), 0.005, int(k[qi]))
            kk = int(k[qi])
            check_topk_row(ids[qi, :kk], dists[qi, :kk], r, f"{w.name} q{qi} k={kk}")
            assert np.all(ids[qi, kk:] == -1) and np.all(np.isinf(dists[qi, kk:]))


def check_topk_row(gi, gd, r, label):
    from gpu_parity import check_topk
    cand_d = np.full(int(r["sc"].size), np.inf)
    cand_d[r["cand"]] = r["cand_d32"]
    check_topk(gi, gd, r["ids"], r["d32"], cand_d, label)


def test_batched_clamps_bad_budgets(taco_mod, tiny):
    import torch
    t = taco_mod
    idx = t.Index(tiny["path"], 0)
    q = torch.from_numpy(tiny["Q"][:4]).cuda()
    alpha = torch.tensor([0.05, 0.0, 2.0, float("nan")], dtype=torch.float64, device="cuda")
    k = torch.tensor([10, 0, 10, 11], dtype=torch.int32, device="cuda")
    ids, _ = idx.search_batched(q, alpha, k, 10, 0.005)
    torch.cuda.synchronize()
    assert idx.device_errors() & 2
    assert idx.device_errors() == 0  # cleared by the read
    assert ids.shape == (4, 10)
    with pytest.raises(t.TacoError):
        idx.search_batched(q, alpha, k, 1025, 0.005)
    idx.close()


def test_graph_replays_match_eager(taco_mod, tiny):
    """A captured search graph replayed several times, with eager work and
    synchronizations between replays, gives the eager results every time, and
    reads the current contents of its input buffers."""
    import torch
    t = taco_mod
    Q = tiny["Q"]
    idx = t.Index(tiny["path"], 0)
    q = torch.from_numpy(Q[:50]).cuda()
    alpha = torch.from_numpy(synthdata.query_budgets(50, 9)[0]).cuda()
    kk = torch.full((50,), 10, dtype=torch.int32, device="cuda")
    e_ids, e_d = idx.search(q, 10, 0.05, 0.005)
    b_ids, b_d = idx.search_batched(q, alpha, kk, 10, 0.005)
    torch.cuda.synchronize()
    e_ids, e_d, b_ids, b_d = (x.clone() for x in (e_ids, e_d, b_ids, b_d))
    idx.set_option(t.TC_OPT_GRAPH, 1)
    ids = torch.empty((50, 10), dtype=torch.int64, device="cuda")
    dists = torch.empty((50, 10), dtype=torch.float32, device="cuda")
    for rep in range(4):
        ids.fill_(-7)
        idx.search(q, 10, 0.05, 0.005, ids=ids, dists=dists)
        torch.cuda.synchronize()
        assert torch.equal(ids, e_ids) and torch.equal(dists, e_d), rep
        _ = (q * 2.0).sum().item()  # eager work between replays
    for rep in range(3):
        ids.fill_(-7)
        idx.search_batched(q, alpha, kk, 10, 0.005, ids=ids, dists=dists)
        torch.cuda.synchronize()
        assert torch.equal(ids, b_ids) and torch.equal(dists, b_d), rep
    # same pointers, new contents: the graph must read the new queries
    q2 = torch.from_numpy(Q[50:100]).cuda()
    idx.set_option(t.TC_OPT_GRAPH, 0)
    e2_ids, e2_d = idx.search(q2, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    idx.set_option(t.TC_OPT_GRAPH, 1)
    idx.search(q, 10, 0.05, 0.005, ids=ids, dists=dists)
    q.copy_(q2)
    idx.search(q, 10, 0.05, 0.005, ids=ids, dists=dists)
    torch.cuda.synchronize()
    assert torch.equal(ids, e2_ids) and torch.equal(dists, e2_d)
    assert idx.device_errors() == 0
    idx.close()


def test_autotune_keeps_results_and_caches(taco_mod, tiny, tmp_path):
    import torch
    t = taco_mod
    idx = t.Index(tiny["path"], 0)
    q = torch.from_numpy(tiny["Q"]).cuda()
    ref_ids, ref_d = idx.search(q, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    ref_ids, ref_d = ref_ids.clone(), ref_d.clone()
    cache = str(tmp_path / "tune.jsonl")
    rep = idx.autotune(q, 10, 0.05, 0.005, cache_path=cache)
    print(rep, flush=True)
    assert "best" in rep
    ids, d = idx.search(q, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    assert torch.equal(ids, ref_ids) and torch.equal(d, ref_d)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"W"' in lines[0]
    idx2 = t.Index(tiny["path"], 0)
    rep2 = idx2.autotune(q, 10, 0.05, 0.005, cache_path=cache)
    assert rep2.startswith("cached")
    ids2, d2 = idx2.search(q, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    assert torch.equal(ids2, ref_ids) and torch.equal(d2, ref_d)
    idx.close()
    idx2.close()


@pytest.mark.parametrize("w", scaled_workloads(), ids=lambda w: w.name)
def test_codes_and_fused_modes_workload_shapes(taco_mod, w):
    """The point-major count (Ns = 8 and 16, up to 4,096 cells) and the
    fused count with its work queue match the split form bit for bit on the
    workload shapes, with uniform and per-query budgets and the fixed-budget
    rule."""
    import torch
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    q = torch.from_numpy(Q).cuda()
    alpha, k = _batched_inputs(w, Q.shape[0])
    ad, kd = torch.from_numpy(alpha).cuda(), torch.from_numpy(k).cuda()
    ref = None
    for mode in (t.TC_COUNT_SPLIT, t.TC_COUNT_CODES, t.TC_COUNT_FUSED):
        idx = t.Index(path, 0)
        try:
            idx.set_option(t.TC_OPT_COUNT_MODE, mode)
        except t.TacoError:
            idx.close()
            assert mode == t.TC_COUNT_FUSED
            continue
        out = []
        for rule in (t.TC_RULE_PRINTED, t.TC_RULE_FIXED):
            idx.set_option(t.TC_OPT_SELECT_RULE, rule)
            i1, d1 = idx.search(q, 10, 0.03, 0.005)
            i2, d2 = idx.search_batched(q, ad, kd, 100, 0.005)
            torch.cuda.synchronize()
            out += [i1.cpu().numpy(), d1.cpu().numpy().view(np.uint32), i2.cpu().numpy(),
                    d2.cpu().numpy().view(np.uint32)]
        assert idx.device_errors() == 0
        idx.close()
        print(f"[{w.name}] mode {mode}", flush=True)
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b), (w.name, mode)


def test_autotune_key_separates_forms_and_batched_tuner(taco_mod, tiny, tmp_path):
    """The tuning cache keys on the options that change which kernels run:
    another selection rule or centroid-distance form measures afresh instead
    of reusing the entry.  The batched tuner keeps tc_search_batched's
    results and caches under its budgets' hash; with TC_OPT_TUNE_PRECISION
    = 0 the re-rank precision stays as set."""
    import torch
    t = taco_mod
    cache = str(tmp_path / "tune.jsonl")
    q = torch.from_numpy(tiny["Q"]).cuda()
    idx = t.Index(tiny["path"], 0)
    assert "best" in idx.autotune(q, 10, 0.05, 0.005, cache_path=cache)
    idx.set_option(t.TC_OPT_SELECT_RULE, t.TC_RULE_PROSE)
    assert "best" in idx.autotune(q, 10, 0.05, 0.005, cache_path=cache)
    idx.set_option(t.TC_OPT_CDIST_PRECISION, t.TC_CDIST_FP8)
    assert "best" in idx.autotune(q, 10, 0.05, 0.005, cache_path=cache)
    assert idx.autotune(q, 10, 0.05, 0.005, cache_path=cache).startswith("cached")
    idx.close()
    assert len(open(cache).read().strip().splitlines()) == 3
    alpha_h, k_h = _batched_inputs(tiny["w"], q.shape[0])
    alpha, k = torch.from_numpy(alpha_h).cuda(), torch.from_numpy(k_h).cuda()
    ref = t.Index(tiny["path"], 0)
    r_ids, r_d = ref.search_batched(q, alpha, k, 100, 0.005)
    torch.cuda.synchronize()
    ref.close()
    idx = t.Index(tiny["path"], 0)
    idx.set_option(t.TC_OPT_PRECISION, t.TC_BF16)
    idx.set_option(t.TC_OPT_TUNE_PRECISION, 0)
    rep = idx.autotune_batched(q, alpha, k, 100, 0.005, cache_path=cache)
    print(rep, flush=True)
    assert "best" in rep and all("precision=1" in ln for ln in rep.strip().splitlines())
    ids, d = idx.search_batched(q, alpha, k, 100, 0.005)
    torch.cuda.synchronize()
    assert torch.equal(ids, r_ids) and torch.equal(d, r_d)
    assert idx.autotune_batched(q, alpha, k, 100, 0.005, cache_path=cache).startswith("cached")
    idx.close()


# ---------------------------------------------------------------------------
# The fixed-budget rule (SuCo's selection, contrasted with Alg 5 in Section
# 4.3): exactly floor(beta*n) candidates, the highest SC-scores, ties by id.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,beta", [
    (0.05, 0.005), (0.01, 0.02), (0.2, 0.001),
    (0.05, 0.0),     # R = 0: no candidates, results padded
    (0.003, 0.5),    # the boundary level is 0: unprobed points in id order
    (1.0, 1.0)])     # every point at level Ns, all taken
def test_tiny_fixed_budget_rule(taco_mod, tiny, alpha, beta):
    print(f"[tiny] fixed budget alpha={alpha} beta={beta}", flush=True)
    _run_all(taco_mod, tiny["path"], tiny["oidx"], tiny["Q"], 10, alpha, beta, 2,
             f"tiny fixed a={alpha} b={beta}")


def _fixed_on_lists(t, path, oidx, Q, alpha, beta, label, options=()):
    """The fixed-budget rule with the list form at list levels 1, 3 and Ns
    (at Ns most queries' boundary level lies below the lists and they are
    queued, counted again and selected on their packed counts): candidates
    against the oracle, once with every stage dumped (the count launch then
    adds every level count) and once with the candidates only (the lists'
    own histogram, exact at the list level and above)."""
    rule = ((t.TC_OPT_SELECT_RULE, t.TC_RULE_FIXED), (t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST))
    for level in (1, 3, oidx.Ns):
        opts = rule + tuple(options) + ((t.TC_OPT_LIST_LEVEL, level),)
        print(f"[{label}] fixed budget on the lists, level {level}", flush=True)
        _run_all(t, path, oidx, Q, 10, alpha, beta, 2, f"{label} lists lvl {level}", options=opts[1:])
        idx = t.Index(path, 0)
        try:
            for opt, val in opts:
                idx.set_option(opt, val)
            g = gpu_search(idx, Q, 10, alpha, beta, ("ncand", "cand"))
        finally:
            idx.close()
        for qi in range(Q.shape[0]):
            compare_query(g, qi, oidx.query(Q[qi], alpha, beta, 10, rule=2), oidx.Ns, 10,
                          f"{label} lists lvl {level} (candidates only)")


def test_fixed_budget_rule_on_the_lists(taco_mod, tiny):
    """The rule on the list form (the first ids of the boundary level found
    on the lists), on the lists' queue, and in a captured graph, stage by
    stage against the oracle; the exact 8-bit re-rank on the lists and the
    graph give the split form's FP32 results bit for bit."""
    t = taco_mod
    rule = ((t.TC_OPT_SELECT_RULE, t.TC_RULE_FIXED),)
    _fixed_on_lists(t, tiny["path"], tiny["oidx"], tiny["Q"], 0.05, 0.005, "tiny")
    print("[tiny] fixed budget in a graph", flush=True)
    _run_all(t, tiny["path"], tiny["oidx"], tiny["Q"], 10, 0.05, 0.005, 2, "tiny fixed graph",
             options=((t.TC_OPT_GRAPH, 1),))
    ref = _search_bits(t, tiny["path"], tiny["Q"], 0.05, rule + ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_SPLIT),))
    for level in (0, 1, 3):
        got = _search_bits(t, tiny["path"], tiny["Q"], 0.05,
                           rule + ((t.TC_OPT_COUNT_MODE, t.TC_COUNT_LIST), (t.TC_OPT_LIST_LEVEL, level),
                                   (t.TC_OPT_PRECISION, t.TC_U8)),
                           calls=2, graph=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), level


def test_fixed_budget_rule_many_tiles(taco_mod):
    w = synthdata.WORKLOADS["gmm-int-1m-d128"].scaled("gmm-int-140k-d128", n=140_000, nq=16)
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    print(f"[{w.name}] fixed budget, many tiles", flush=True)
    for beta in (0.005, 0.05):
        _run_all(taco_mod, path, oidx, Q, 10, 0.05, beta, 2, f"140k fixed b={beta}",
                 options=((taco_mod.TC_OPT_TILE_IDS, 8192),))
    # 137 tiles of 1024 ids: the lists' tile counts are scanned 128 tiles at a time
    _fixed_on_lists(taco_mod, path, oidx, Q, 0.05, 0.005, "140k", options=((taco_mod.TC_OPT_TILE_IDS, 1024),))
