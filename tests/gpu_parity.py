"""Helpers that run the GPU path and compare it with the oracle, stage by
stage (imported by the GPU tests; no tests here)."""
import os

import numpy as np

import synthdata
from oracle import oracle as O

DIST_RTOL = 1e-5  # FP32 re-rank distances: GPU vs the oracle's FP32 chain


def cache_dir():
    d = os.environ.get("TACO_CACHE") or os.path.join(
        os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".taco_cache")
    os.makedirs(d, exist_ok=True)
    return d


def workload_index(w, X=None):
    """Path of the oracle-built index of workload ``w`` (built once, cached
    under the workload's name, which encodes its recipe and sizes)."""
    path = os.path.join(cache_dir(), f"{w.name}-n{w.n}-s{w.seed:x}.tcx")
    if not os.path.exists(path):
        tmp = path + ".tmp%d" % os.getpid()
        O.build_workload_index(w, tmp, X)
        os.replace(tmp, path)
    return path


def gpu_search(idx, Q, k, alpha, beta, fields=None):
    """Run the GPU search with stage dumps; returns numpy arrays."""
    import torch
    q = torch.from_numpy(np.ascontiguousarray(Q)).to(f"cuda:{idx.device}")
    dump = idx.dump_buffers(Q.shape[0], fields) if fields else None
    if dump is None:
        ids, dists = idx.search(q, k, alpha, beta)
    else:
        ids, dists = idx.search_debug(q, k, alpha, beta, dump)
    torch.cuda.synchronize()
    assert idx.device_errors() == 0, "a fused count/select wait timed out"
    out = {f: t.cpu().numpy() for f, t in (dump or {}).items()}
    out["ids"], out["dists"] = ids.cpu().numpy(), dists.cpu().numpy()
    return out


def check_topk(g_ids, g_d, o_ids, o_d, cand_d=None, label=""):
    """Result ids must match the oracle except at distance ties inside the
    FP32 tolerance; distances within DIST_RTOL of the oracle's."""
    k = len(o_ids)
    valid = o_ids >= 0
    assert np.array_equal(g_ids < 0, ~valid), f"{label}: padding differs"
    assert np.all(np.isinf(g_d[~valid])), f"{label}: padded distances must be +inf"
    od, gd = o_d[valid].astype(np.float64), g_d[valid].astype(np.float64)
    assert np.all(np.abs(gd - od) <= DIST_RTOL * np.abs(od) + 1e-30), f"{label}: distances differ"
    assert np.all(np.diff(gd) >= 0), f"{label}: GPU results not ascending"
    if not np.array_equal(g_ids, o_ids):
        kth = od[-1]
        diff = set(g_ids[valid].tolist()) ^ set(o_ids[valid].tolist())
        assert cand_d is not None, f"{label}: ids differ {g_ids} vs {o_ids}"
        for i in diff:
            di = float(cand_d[int(i)])
            assert abs(di - kth) <= 2 * DIST_RTOL * kth, f"{label}: id {i} differs beyond a tie"


def compare_query(g, qi, r, Ns, k, label):
    """Compare GPU dumps of query qi with the oracle's dump r."""
    lab = f"{label} q{qi}"
    if "qt" in g:
        assert np.array_equal(g["qt"][qi].view(np.uint32), r["qt"].view(np.uint32)), f"{lab}: q' bits"
    if "cdist" in g:
        assert np.array_equal(g["cdist"][qi].view(np.uint32), r["cdist"].view(np.uint32)), \
            f"{lab}: half-centroid distance bits"
    if "corder" in g:
        assert np.array_equal(g["corder"][qi], r["corder"]), f"{lab}: centroid order"
    if "ncells" in g:
        assert np.array_equal(g["ncells"][qi], r["ncells"]), f"{lab}: number of probed cells"
    if "cells" in g:
        for j in range(Ns):
            nc = int(r["ncells"][j])
            assert np.array_equal(g["cells"][qi, j, :nc], r["cells"][j]), f"{lab}: probed cells j={j}"
    if "retrieved" in g:
        assert np.array_equal(g["retrieved"][qi], r["retrieved"]), f"{lab}: retrieved"
    if "sc" in g:
        assert np.array_equal(g["sc"][qi], r["sc"]), f"{lab}: collision counts"
    if "hist" in g:
        assert np.array_equal(g["hist"][qi], r["hist"]), f"{lab}: level histogram"
    if "last" in g:
        assert int(g["last"][qi]) == r["last"], f"{lab}: threshold"
    cand_d = None
    if "ncand" in g:
        nc = int(g["ncand"][qi])
        assert nc == r["ncand"], f"{lab}: candidate count"
        if "cand" in g:
            gc = g["cand"][qi, :nc]
            order = np.argsort(gc, kind="stable")
            assert np.array_equal(gc[order], r["cand"]), f"{lab}: candidate set"
            if "cand_dist" in g:
                gdist = g["cand_dist"][qi, :nc][order].astype(np.float64)
                od = r["cand_d32"].astype(np.float64)
                assert np.all(np.abs(gdist - od) <= DIST_RTOL * np.abs(od) + 1e-30), \
                    f"{lab}: candidate distances"
                cand_d = np.full(int(r["sc"].size), np.inf)
                cand_d[r["cand"]] = od
    check_topk(g["ids"][qi], g["dists"][qi], r["ids"], r["d32"], cand_d, lab)


ALL_STAGES = ("qt", "cdist", "corder", "cells", "ncells", "retrieved", "sc", "hist", "last",
              "ncand", "cand", "cand_dist")


def scaled_workloads():
    """The four larger recipes at sizes the oracle builds in seconds, with
    index shapes (d, Ns, s, l) kept; n chosen to span several LDS tiles."""
    W = synthdata.WORKLOADS
    return [
        W["gmm-int-1m-d128"].scaled("gmm-int-40k-d128", n=40_000, nq=24),
        W["aniso-1m-d960"].scaled("aniso-12k-d960", n=12_000, nq=12, iters=8),
        W["sphere-10m-d96"].scaled("sphere-50k-d96", n=50_000, nq=24, n_train=None),
        W["zipf-1m-d256"].scaled("zipf-30k-d256", n=30_000, nq=24),
    ]
