"""Throughput of the TaCo query stage on one MI355X.

One step = one pass of the whole query path (transform, centroid distances,
probe, collision count, candidate selection, re-rank, top-k) over one batch of
queries already resident in HBM.  The default workload is the 10M x 96
L2-normalised Gaussian mixture (4,096 components, angular spread 0.3 rad),
Ns = 8 subspaces of 12 dims, 64 x 64 IMI cells per subspace, 10,000 queries,
k = 10: the largest configuration that fits one GPU.  The value is QPS at
recall@10 = 0.95 of the reduced-precision batched path (FP8 e4m3 centroid
distances with per-subspace scales, BF16 re-rank with an FP32 re-check,
autotuned launch shapes, one batch per step replayed as a captured HIP
graph), read off the Pareto frontier of an (alpha, beta) sweep; the plain
FP32 path (default options, eager launches) is reported beside it.

Recall is tie-aware against FP64 k-th neighbour distances of a sample of the
queries: a shortlist from the FP64 expansion |x|^2 - 2 x.q computed with
torch on the GPU (a library GEMM, not this project's kernels), then exact FP64
distances of the shortlist on the host.

Legs:
  * the oracle (test infrastructure) builds the serialized index from the
    workload's seed; both the GPU and the oracle search that file.  Its query
    is timed on a bounded sample on all host threads and on one thread
    (cpu_baseline).
  * GPU paths, per sweep point: "fp32" (defaults: split counting, FP32
    centroid distances and re-rank, eager launches), "fp32_tuned" (FP32
    everywhere, autotuned launch shapes, one batch per step, graph replay),
    "tuned" (the autotuner also picks the exact re-rank form: FP32, BF16 or
    8-bit rows with an FP32 re-check), "bf16" (BF16 centroid distances on the
    matrix cores, BF16 re-rank) and "fp8" (FP8 centroid distances, BF16
    re-rank).  Per-kernel times come from HIP events on the search stream
    during an eager run; the graph paths' QPS is the replay rate.
  * precision report: relative error of the BF16 / FP8 centroid distances
    against FP64, recall loss of each path against FP32 at every sweep point,
    and the fraction of candidates the BF16 re-rank re-checks in FP32.
  * GPU index build (Alg 1-3) of the same workload, beside the oracle's.

``--workload zipf-1m-d256`` runs the batched configuration instead: 100,000
queries with per-query alpha (log-uniform in [0.005, 0.1]) and k in
{1, 10, 100}, one tc_search_batched call per step, against per-query launches
and the FP32 plain path, swept over beta.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthdata  # noqa: E402

DEFAULT_WORKLOAD = "sphere-10m-d96"
METRIC = "QPS at recall@10=0.95 on 1 MI355X; BF16/FP8+batched vs FP32 plain"
RECALL_TARGET = 0.95
HBM_PEAK_GBS = 8000.0
KERNELS = ("transform", "cdist", "probe", "count", "select", "rerank", "topk", "recheck", "count_select", "stream")

# Per workload: the (alpha, beta) sweep, the paths run, the one the value is
# read from, and the oracle's sweep points (a bounded sample near the target).
PLANS = {
    "sphere-10m-d96": dict(
        sweep=[(0.002, b) for b in (0.0001, 0.0002, 0.00025, 0.0003)], tune_at=(0.002, 0.0002),
        paths=("fp32", "fp32_tuned", "bf16", "fp8"), main="fp8",
        cpu_points=[(0.002, b) for b in (0.0002, 0.00025, 0.0003)], cpu_sample=4000),
    "gmm-int-1m-d128": dict(
        sweep=[(0.05, b) for b in (0.0001, 0.0002, 0.0005, 0.001, 0.005)], tune_at=(0.05, 0.0005),
        paths=("fp32", "tuned", "bf16", "fp8"), main="fp8",
        cpu_points=[(0.05, b) for b in (0.0001, 0.0002, 0.0005, 0.001)], cpu_sample=4000),
    "aniso-1m-d960": dict(
        sweep=[(a, b) for a in (0.1, 0.2, 0.3) for b in (0.01, 0.02, 0.05)], tune_at=(0.2, 0.05),
        paths=("fp32", "fp32_tuned", "bf16"), main="bf16",
        cpu_points=[(0.2, b) for b in (0.02, 0.05)], cpu_sample=400),
    "zipf-1m-d256": dict(
        betas=(0.005, 0.01, 0.02, 0.05, 0.15), tune_beta=0.05, paths=("fp32", "batched"), main="batched",
        per_query_sample=2000, cpu_points=[(None, b) for b in (0.02, 0.15)], cpu_sample=2000),
}

# path -> (centroid-distance form, re-rank precision or None to let the
# tuner choose an exact form, tuned/graph/one-batch, selection rule)
PATHS = {
    "fp32": ("fp32", "fp32", False, "printed"),
    "fp32_tuned": ("fp32", "fp32", True, "printed"),
    "tuned": ("fp32", None, True, "printed"),
    "bf16": ("bf16", "bf16", True, "printed"),
    "fp8": ("fp8", "bf16", True, "printed"),
    # the fixed budget of the floor(beta*n) highest SC-scores (SuCo's
    # selection, contrasted with Alg 5 in Section 4.3) on the fp8 path's
    # options; not in any plan's default paths
    "fp8_fixed": ("fp8", "bf16", True, "fixed"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# cpu_baseline leg: everything that runs the oracle lives here
# ---------------------------------------------------------------------------

def cpu_baseline_index(w, X):
    """Serialized index built by the oracle from the workload seed (cached).
    Returns (path, seconds the oracle's build took, or None when cached)."""
    from oracle import oracle as O
    cache = os.environ.get("TACO_CACHE") or os.path.join(ROOT, ".taco_cache")
    os.makedirs(cache, exist_ok=True)
    path = os.path.join(cache, f"{w.name}-n{w.n}-s{w.seed:x}.tcx")
    built_s = None
    if not os.path.exists(path):
        t = time.time()
        tmp = path + ".tmp%d" % os.getpid()
        O.build_workload_index(w, tmp, X)
        os.replace(tmp, path)
        built_s = time.time() - t
        log(f"oracle built the index in {built_s:.1f}s on {O.max_threads()} threads -> {path}")
    return path, built_s


def cpu_baseline_build_time(w, X):
    """Seconds the oracle takes to build the workload's index (into a
    scratch file, removed afterwards)."""
    from oracle import oracle as O
    import tempfile
    fd, tmp = tempfile.mkstemp(suffix=".tcx")
    os.close(fd)
    try:
        t = time.time()
        O.build_workload_index(w, tmp, X)
        dt = time.time() - t
    finally:
        os.unlink(tmp)
    log(f"oracle built the index in {dt:.1f}s on {O.max_threads()} threads (timing only)")
    return dt


def cpu_baseline_timing(path, X, Q, w, gt, points, sample, threads, alpha_q=None, k_q=None):
    """The oracle as it stands, parallel over queries with OpenMP on
    `threads` host threads, timed on the first `sample` queries at each
    (alpha, beta) of `points` (one warm-up batch first); its recall is read
    on the queries that have ground truth."""
    from oracle import oracle as O
    oidx = O.OracleIndex(path)
    pts = []
    Qs = Q[:sample]
    S = min(sample, gt["n"])
    kk = w.k if k_q is None else int(k_q.max())
    for a, b in points:
        av = a if alpha_q is None else alpha_q[:sample]
        oidx.query_batch(Qs[:threads], av if np.isscalar(av) else av[:threads], b, kk, nthreads=threads)
        t = time.time()
        ids = oidx.query_batch(Qs, av, b, kk, nthreads=threads)
        dt = time.time() - t
        rec = recall_of(ids[:S], gt, X, Qs[:S], w.k, None if k_q is None else k_q[:S])
        pts.append(dict(alpha=a, beta=b, qps=sample / dt, recall=rec, seconds=dt))
        log(f"oracle alpha={a} beta={b}: {sample / dt:.1f} QPS on {threads} threads over {sample} "
            f"queries, recall {rec:.4f}")
    oidx.close()
    return pts


# ---------------------------------------------------------------------------
# ground truth and recall
# ---------------------------------------------------------------------------

def ground_truth(X, Qs, ks, dev, chunk=64):
    """FP64 distance of each query's k-th nearest base row for every k in
    `ks`: a shortlist of max(ks)+32 rows by the FP64 expansion
    |x|^2 - 2 x.q (torch on the GPU), then the exact FP64 sum of squared
    differences on the shortlist, sorted, on the host."""
    import torch
    kmax = max(ks)
    m = min(kmax + 32, X.shape[0])
    out = {k: np.empty(Qs.shape[0]) for k in ks}
    Xd = torch.from_numpy(X).to(dev)
    xn = torch.empty(X.shape[0], dtype=torch.float64, device=dev)
    step = 1 << 20
    for r0 in range(0, X.shape[0], step):
        xn[r0:r0 + step] = (Xd[r0:r0 + step].double() ** 2).sum(1)
    for c0 in range(0, Qs.shape[0], chunk):
        q = torch.from_numpy(Qs[c0:c0 + chunk]).to(dev).double()
        best = None
        for r0 in range(0, X.shape[0], step):
            dd = xn[r0:r0 + step][None, :] - 2.0 * (q @ Xd[r0:r0 + step].double().T)
            v, i = torch.topk(dd, min(m, dd.shape[1]), dim=1, largest=False)
            i = i + r0
            if best is None:
                best = (v, i)
            else:
                vv, ii = torch.cat([best[0], v], 1), torch.cat([best[1], i], 1)
                v2, j = torch.topk(vv, m, dim=1, largest=False)
                best = (v2, torch.gather(ii, 1, j))
        short = best[1].cpu().numpy()
        for i in range(short.shape[0]):
            d = np.sort(((X[short[i]].astype(np.float64) - Qs[c0 + i].astype(np.float64)) ** 2).sum(1))
            for k in ks:
                out[k][c0 + i] = d[k - 1]
    del Xd, xn
    torch.cuda.empty_cache()
    return out


def recall_at_k(ids, kth, X, Qs, k):
    """Mean recall@k (Section 5.1), tie-aware: a returned id is a true
    neighbour when its FP64 distance is at most the k-th true distance (up
    to 1e-12 relative, for summation-order differences)."""
    hits = 0
    for i in range(ids.shape[0]):
        r = ids[i, :k]
        r = r[r >= 0]
        if r.size:
            d = ((X[r].astype(np.float64) - Qs[i].astype(np.float64)) ** 2).sum(1)
            hits += int(np.count_nonzero(d <= kth[i] * (1.0 + 1e-12)))
    return hits / float(ids.shape[0] * k)


def recall_of(ids, gt, X, Qs, k, k_q=None):
    """recall@k, or for per-query k: recall@10 over the queries asking for at
    least 10 results (their first 10) and recall@1 over those asking for 1,
    averaged by query."""
    if k_q is None:
        return recall_at_k(ids, gt[k], X, Qs, k)
    big, one = k_q >= 10, k_q == 1
    m = len(k_q)  # the ground truth may cover more queries than this sample
    tot = 0.0
    if big.any():
        tot += recall_at_k(ids[big], gt[10][:m][big], X, Qs[big], 10) * big.sum()
    if one.any():
        tot += recall_at_k(ids[one], gt[1][:m][one], X, Qs[one], 1) * one.sum()
    return tot / float(big.sum() + one.sum())


def index_centroids(path):
    """The half-subspace centroids C1 [Ns][l][h1], C2 [Ns][l][h2] read from
    the index file (128-byte header, then mean, B, C1, C2, all f32)."""
    hdr = np.fromfile(path, dtype=np.uint8, count=128)
    d, Ns, s, h1, h2, l = (int(v) for v in hdr[24:48].view(np.int32))
    off = 128 + 4 * (d + d * Ns * s)
    c1 = np.fromfile(path, dtype=np.float32, count=Ns * l * h1, offset=off).reshape(Ns, l, h1)
    c2 = np.fromfile(path, dtype=np.float32, count=Ns * l * h2, offset=off + 4 * Ns * l * h1).reshape(Ns, l, h2)
    return c1, c2


def cdist_errors(taco, idx, qd, w, alpha, beta, c1, c2, nq_err=200):
    """Relative error of the BF16 and FP8 centroid distances (matrix cores)
    and of the FP32 chain against FP64 distances of the same FP32 transformed
    queries and FP32 centroids, over every half-subspace centroid."""
    import torch
    Ns, l, h1 = c1.shape
    rep = {}
    P = min(nq_err, qd.shape[0])
    for name, val in (("fp32", taco.TC_CDIST_FP32), ("bf16", taco.TC_CDIST_BF16), ("fp8", taco.TC_CDIST_FP8)):
        idx.set_option(taco.TC_OPT_CDIST_PRECISION, val)
        dump = idx.dump_buffers(P, ("qt", "cdist"))
        idx.search_debug(qd[:P], w.k, alpha, beta, dump)
        torch.cuda.synchronize()
        qt = dump["qt"].cpu().numpy().astype(np.float64)
        cd = dump["cdist"].cpu().numpy().astype(np.float64)
        s = qt.shape[1] // Ns
        rel = []
        for j in range(Ns):
            for h, (cen, lo, hi) in enumerate(((c1[j], 0, h1), (c2[j], h1, s))):
                x = qt[:, j * s + lo:j * s + hi]
                ex = ((x[:, None, :] - cen[None, :, :].astype(np.float64)) ** 2).sum(2)
                m = ex > 0
                rel.append(np.abs(cd[:, j, h, :][m] - ex[m]) / ex[m])
        rel = np.concatenate(rel)
        rep[name] = dict(rel_err_max=float(rel.max()), rel_err_mean=float(rel.mean()),
                         rel_err_p99=float(np.quantile(rel, 0.99)))
    idx.set_option(taco.TC_OPT_CDIST_PRECISION, taco.TC_CDIST_FP32)
    rep["sample"] = f"first {P} queries, every half-subspace centroid"
    return rep


def recheck_fraction(taco, idx, qd, w, alpha, beta):
    """Fraction of the candidates the BF16 re-rank recomputes in FP32."""
    import torch
    idx.set_option(taco.TC_OPT_PRECISION, taco.TC_BF16)
    P = min(2000, qd.shape[0])
    dump = idx.dump_buffers(P, ("ncand", "nrecheck"))
    idx.search_debug(qd[:P], w.k, alpha, beta, dump)
    torch.cuda.synchronize()
    return float(dump["nrecheck"].sum().item()) / max(1.0, float(dump["ncand"].sum().item()))


def qps_at_recall(points, target=RECALL_TARGET):
    """QPS at the target recall from (recall, qps) points: the Pareto
    frontier (no other point has both higher recall and higher QPS), sorted
    by recall, is read at the target -- the best QPS of a frontier point at
    or above it, else None if no point reaches it, and where the frontier
    steps across the target, the linear interpolation between the two
    neighbouring frontier points if that is higher."""
    front = [p for p in points
             if not any(o["recall"] >= p["recall"] and o["qps"] >= p["qps"] and
                        (o["recall"] > p["recall"] or o["qps"] > p["qps"]) for o in points)]
    front.sort(key=lambda p: p["recall"])
    above = [p for p in front if p["recall"] >= target]
    if not above:
        return None
    best = max(p["qps"] for p in above)
    below = [p for p in front if p["recall"] < target]
    if below:
        lo, hi = below[-1], above[0]
        f = (hi["recall"] - target) / (hi["recall"] - lo["recall"])
        best = max(best, hi["qps"] + f * (lo["qps"] - hi["qps"]))
    return best


def code_text(src):
    """C++ source without its comments and with runs of whitespace folded:
    what the compiler sees, so that a comment edit keeps the hash."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "runtime.cpp"):
        with open(os.path.join(ROOT, "paper_2603_24919_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def launch_config(tuned):
    """The launch configuration in a tuner report line ("... W=131072 mode=3
    qpw=8 rr=8 precision=1 cqpw=32 nt=768 ..."): those fields as a dict."""
    import re
    return {k: int(v) for k, v in re.findall(r"\b(W|mode|qpw|rr|precision|cqpw|nt)=(\d+)", tuned or "")}


def traffic_records(path):
    """The records of a traffic summary file (one per launch configuration)."""
    if not os.path.exists(path):
        return []
    try:
        doc = json.load(open(path))
    except ValueError:
        return []
    return doc.get("records", [doc] if "kernels" in doc else [])


# The launch settings each kernel's own work depends on (the others change
# only which kernels run beside it); kernels not listed need all of them.
TRAFFIC_KEYS = {
    "count": ("W", "mode", "nt", "cqpw"), "count_select": ("W", "mode", "nt", "cqpw"),
    "rerank": ("W", "mode", "precision", "rr"), "recheck": ("W", "mode", "precision", "rr"),
}


def traffic_from_profiles(workload, kernel, tuned=None, path=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload: the record taken on the current kernel sources,
    on the same bench path (when `path` is given: its precision forms and
    selection rule), whose launch configuration agrees with the run's
    (`tuned`, its tuner report) in every setting the kernel depends on, else
    None."""
    keys = TRAFFIC_KEYS.get(kernel, ("W", "mode", "qpw", "rr", "precision", "cqpw", "nt"))
    run = launch_config(tuned)
    want = {k: run.get(k) for k in keys}
    for rec in traffic_records(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")):
        if rec.get("source_hash") != source_hash() or rec.get("workload") != workload:
            continue
        if path is not None and rec.get("path") != path:
            continue
        have = launch_config(rec.get("tuned_config"))
        if not run or {k: have.get(k) for k in keys} != want:
            continue
        k = rec.get("kernels", {}).get(kernel)
        return None if k is None else k.get("hbm_bytes_per_launch")
    return None


def algorithmic_bytes(idx, q, w, alpha, beta, precision, alpha_dev=None, k_dev=None, k_max=None):
    """Bytes the method must move, per kernel, for one step, at the per-query
    figures of a stage-count pass: count: ids of the probed lists (4 B each)
    + the slice bounds and probed cell ids (12 B per probed cell); select:
    the candidate ids written (4 B) and the probed cells read; rerank: each
    candidate's row (4d B; 2d B plus its 4 B error bound in BF16; d B plus a
    12 B record in 8 bits), id and distance (8 B) plus the query (4d B);
    topk: candidate keys (8 B each) and the output (12k B); recheck: the
    candidates' lower bounds (4 B each).  Returns (bytes per kernel, per-query
    averages, total increments)."""
    import torch
    nq = q.shape[0]
    if alpha_dev is None:
        dump = idx.dump_buffers(nq, ("retrieved", "ncells", "ncand"))
        idx.search_debug(q, w.k, alpha, beta, dump)
        torch.cuda.synchronize()
        R = float(dump["retrieved"].sum().item())
        P = float(dump["ncells"].sum().item())
        C = float(dump["ncand"].sum().item())
    else:
        # per-query budgets: each query's stages equal those of a search with
        # its own alpha, so a sample of queries searched one by one gives the
        # per-query averages, scaled to the batch
        a_h, k_h = alpha_dev.cpu().numpy(), k_dev.cpu().numpy()
        m = min(nq, 256)
        R = P = C = 0.0
        for i in range(m):
            one = idx.dump_buffers(1, ("retrieved", "ncells", "ncand"))
            idx.search_debug(q[i:i + 1], int(k_h[i]), float(a_h[i]), beta, one)
            torch.cuda.synchronize()
            R += float(one["retrieved"].sum().item())
            P += float(one["ncells"].sum().item())
            C += float(one["ncand"].sum().item())
        R, P, C = R * nq / m, P * nq / m, C * nq / m
    d = w.d
    kk = w.k if k_max is None else k_max
    row = {"fp32": 4.0 * d, "bf16": 2.0 * d + 4.0, "u8": d + 12.0}[precision]
    return dict(
        transform=nq * (4.0 * d + 4.0 * w.M),
        probe=nq * w.M * 4.0 + 4.0 * P,
        count=4.0 * R + 12.0 * P,
        select=4.0 * C + 4.0 * P,
        count_select=4.0 * R + 16.0 * P + 4.0 * C,
        rerank=C * (row + 8.0) + nq * 4.0 * d,
        topk=8.0 * C + 12.0 * kk * nq,
        recheck=4.0 * C,
    ), dict(retrieved=R / nq, probed_cells=P / nq, candidates=C / nq), R


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def gpu_build_leg(taco, torch, w, X, dev, reps):
    """Alg 1-3 on the GPU from the base already resident in HBM: the
    library's HIP-event times of each stage (statistics, eigensolver, Alg 2
    and uploads, transform, k-means, IMI); one warm-up build, then the
    fastest of ``reps``."""
    xb = torch.from_numpy(X).to(dev)
    train, init = synthdata.kmeans_seeding(w)
    runs = []
    for r in range(reps + 1):
        idx = taco.Index.build(xb, w.Ns, w.s, w.l, w.iters, init, train, w.seed)
        ms = np.array(idx.stage_ms, dtype=float)
        idx.close()
        if r:
            runs.append(ms)
    del xb
    torch.cuda.empty_cache()
    best = min(runs, key=lambda m: float(m.sum()))
    return dict(workload=w.name, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l, kmeans_iters=w.iters,
                n_train=w.n_train, gpu_ms=float(best.sum()),
                stages_ms=dict(zip(BUILD_STAGES, map(float, best))), reps=reps,
                timing="HIP events around each stage, base resident in HBM; the index's search "
                       "preparation and the host copies excluded")


BUILD_STAGES = ("stats", "eigen", "allocate", "transform", "kmeans", "imi")


def timed_steps(idx, taco, run, stream, steps, warmup, profile=True):
    """Warm-up, then exactly `steps` calls of `run` (one search of the whole
    batch) between two events on the search stream.  Returns (ms, per-kernel
    totals from the library's own HIP events)."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    if profile:
        idx.set_option(taco.TC_OPT_PROFILE, 1)
        idx.profile_reset()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        run()
    stop.record(stream)
    torch.cuda.synchronize()
    kern = {}
    if profile:
        for kname in KERNELS:
            tot, n = idx.kernel_time(kname)
            kern[kname] = dict(ms_total=tot, launches=n)
        idx.set_option(taco.TC_OPT_PROFILE, 0)
    return start.elapsed_time(stop), kern


def configure_path(taco, torch, idx, pname, dev, nq):
    """Options of a path before tuning: its centroid-distance form, its
    re-rank precision (fixed unless the tuner chooses), and for the tuned
    paths one batch per step (scratch up to 60% of the free device memory)."""
    cd, prec, tuned, rule = PATHS[pname]
    idx.set_option(taco.TC_OPT_SELECT_RULE, dict(printed=taco.TC_RULE_PRINTED, fixed=taco.TC_RULE_FIXED)[rule])
    idx.set_option(taco.TC_OPT_CDIST_PRECISION, dict(fp32=taco.TC_CDIST_FP32, bf16=taco.TC_CDIST_BF16,
                                                     fp8=taco.TC_CDIST_FP8)[cd])
    if prec is not None:
        idx.set_option(taco.TC_OPT_PRECISION, dict(fp32=taco.TC_FP32, bf16=taco.TC_BF16)[prec])
        idx.set_option(taco.TC_OPT_TUNE_PRECISION, 0)
    if tuned:
        free, _ = torch.cuda.mem_get_info(dev)
        idx.set_option(taco.TC_OPT_SCRATCH_BYTES, int(free * 0.6))
        idx.set_option(taco.TC_OPT_MAX_BATCH, nq)


def kernel_rates(kern, alg, steps):
    for kname, v in kern.items():
        launches = max(v["launches"], 1)
        v["ms_per_launch"] = v["ms_total"] / launches
        b = alg.get(kname)
        v["alg_bytes_per_launch"] = None if b is None else b * steps / launches
        v["alg_GBps"] = None if (b is None or v["ms_total"] <= 0) else (b * steps) / (v["ms_total"] * 1e-3) / 1e9


def run_point(taco, torch, idx, pname, run, stream, args, w, nq, recall_fn, alg_fn, tuned_cfg, beta, k_max):
    """One sweep point of one path: an eager timed run with per-kernel
    events, then for the tuned paths (already tuned: `tuned_cfg` is their
    configuration) the graph replay rate; recall from the results of the
    timed runs."""
    cd, prec, tuned = PATHS.get(pname, ("fp32", None, True, "printed"))[:3]
    t0 = time.time()
    point = {}
    if tuned:
        point["config"] = tuned_cfg
    ms, kern = timed_steps(idx, taco, run, stream, args.steps, args.warmup)
    rec = recall_fn()
    real_prec = prec
    if real_prec is None:
        cfg = point.get("config", "")
        real_prec = {"0": "fp32", "1": "bf16", "2": "u8"}.get(cfg.split("precision=")[1].split()[0], "fp32") \
            if "precision=" in cfg else "fp32"
    alg, avg, incr = alg_fn(real_prec)
    kernel_rates(kern, alg, args.steps)
    qps = nq * args.steps / (ms * 1e-3)
    point.update(qps=qps, recall=rec, ms_per_step=ms / args.steps, kernels=kern, per_query=avg,
                 increments_per_step=incr, batches_per_step=-(-nq // idx.batch_capacity(beta, k_max)),
                 rerank_precision=real_prec, cdist=cd)
    if tuned:
        idx.set_option(taco.TC_OPT_GRAPH, 1)
        gms, _ = timed_steps(idx, taco, run, stream, args.steps, args.warmup, profile=False)
        grec = recall_fn()
        idx.set_option(taco.TC_OPT_GRAPH, 0)
        point.update(eager_qps=qps, eager_ms_per_step=ms / args.steps,
                     graph_qps=nq * args.steps / (gms * 1e-3), qps=nq * args.steps / (gms * 1e-3),
                     ms_per_step=gms / args.steps, recall=min(rec, grec))
    point["seconds"] = time.time() - t0
    return point


def describe(pname, p):
    ks = ", ".join(f"{k} {v['ms_total'] / max(1, v['launches']):.3f}" for k, v in p["kernels"].items()
                   if v["ms_total"] > 0)
    return (f"{pname}: {p['qps']:,.0f} QPS, {p['ms_per_step']:.3f} ms/step, recall {p['recall']:.4f}, "
            f"|C| {p['per_query']['candidates']:.0f}; {ks}")


def operating_point(sweep):
    """The fastest sweep point at or above the target recall (else the
    highest-recall point)."""
    ok = [p for p in sweep if p["recall"] >= RECALL_TARGET]
    return max(ok, key=lambda p: p["qps"]) if ok else max(sweep, key=lambda p: p["recall"])


def roofline_of(workload, op, path_name):
    """The dominant kernel at the operating point against the HBM peak:
    algorithmic bytes per launch over its mean HIP-event launch time, with
    the counter-measured bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by
    a known-size copy) when a summary of the current sources exists."""
    dom = max(op["kernels"], key=lambda k_: op["kernels"][k_]["ms_total"])
    dk = op["kernels"][dom]
    achieved = dk["alg_GBps"]
    traffic = traffic_from_profiles(workload, dom, op.get("config"), path_name)
    r = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
             frac=None if achieved is None else achieved / HBM_PEAK_GBS, traffic=traffic,
             alg_bytes_per_launch=dk["alg_bytes_per_launch"], ms_per_launch=dk["ms_per_launch"],
             alpha=op.get("alpha"), beta=op.get("beta"), path=path_name)
    if traffic is not None and dk["ms_per_launch"]:
        r["counter_GBps"] = traffic / (dk["ms_per_launch"] * 1e-3) / 1e9
        r["counter_frac"] = r["counter_GBps"] / HBM_PEAK_GBS
    c = op["kernels"].get("count")
    if c and c["ms_total"] > 0 and op.get("steps"):
        # the count kernel's own limiter: one LDS increment per probed id
        r["count_increments_per_s"] = op["increments_per_step"] / (c["ms_total"] / op["steps"] * 1e-3)
    return r


def sclinear_leg(taco, torch, path, qd, Q, X, gt, S, w, op, stream, m):
    """SC-Linear (the index-free baseline of Section 2.3) on the GPU at the
    operating point's alpha and beta, over the first m queries: one warm-up
    call, then one timed call (HIP events); recall on those with ground
    truth.  The paper's Table 2 reports the TaCo / SC-Linear query-time
    ratio the same way."""
    m = min(m, qd.shape[0])
    idx = taco.Index(path, 0)
    q = qd[:m]
    ids = torch.empty((m, w.k), dtype=torch.int64, device=qd.device)
    dists = torch.empty((m, w.k), dtype=torch.float32, device=qd.device)
    a, b = op["alpha"], op["beta"]
    idx.search_sclinear(q, w.k, a, b, ids=ids, dists=dists, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    idx.search_sclinear(q, w.k, a, b, ids=ids, dists=dists, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    Sm = min(S, m)
    rec = recall_at_k(ids[:Sm].cpu().numpy(), gt[w.k][:Sm], X, Q[:Sm], w.k)
    idx.close()
    return dict(qps=m / (ms * 1e-3), ms=ms, recall=rec, alpha=a, beta=b, queries=m,
                note="exact per-subspace collisions over all n points, the floor(beta*n) highest "
                     "SC-scores, FP32 re-rank; one call over the queries")


def strip_point(p):
    return dict({k: p[k] for k in ("alpha", "beta", "qps", "recall", "ms_per_step", "per_query",
                                   "batches_per_step", "rerank_precision", "cdist") if k in p},
                graph_qps=p.get("graph_qps"), eager_qps=p.get("eager_qps"), config=p.get("config"),
                kernels={k_: dict(ms_per_launch=v["ms_per_launch"], launches=v["launches"],
                                  alg_GBps=v["alg_GBps"]) for k_, v in p["kernels"].items() if v["launches"]})


def cpu_baseline_leg(path, X, Q, w, gt, plan, args, alpha_q=None, k_q=None):
    """The oracle on all host threads over a bounded sample at the plan's
    points (value read at the target recall like the GPU's), and on one
    thread at the point nearest the target."""
    from oracle import oracle as O
    threads = O.max_threads()
    cs = min(args.cpu_sample or plan["cpu_sample"], Q.shape[0])
    points = plan.get("cpu_points") or [(None, b) for b in plan["betas"][:2]]
    pts = cpu_baseline_timing(path, X, Q, w, gt, points, cs, threads, alpha_q, k_q)
    near = min(pts, key=lambda p: abs(p["recall"] - RECALL_TARGET))
    one_sample = max(50, cs // max(1, threads) // 2)
    one = cpu_baseline_timing(path, X, Q, w, gt, [(near["alpha"], near["beta"])], one_sample, 1, alpha_q, k_q)[0]
    return dict(value=qps_at_recall(pts), unit="queries/s", cores=threads, kind="oracle",
                sample=f"first {cs} of the {Q.shape[0]} queries at each point "
                       f"{[(p['alpha'], p['beta']) for p in pts]}, OpenMP over queries on {threads} "
                       f"threads, recall on the first {min(cs, gt['n'])}; value read at recall@10="
                       f"{RECALL_TARGET} like the GPU's",
                seconds=sum(p["seconds"] for p in pts),
                points=[dict(alpha=p["alpha"], beta=p["beta"], qps=p["qps"], recall=p["recall"]) for p in pts],
                single_core=dict(cores=1, qps=one["qps"], recall=one["recall"], alpha=one["alpha"],
                                 beta=one["beta"], sample=f"first {one_sample} queries", seconds=one["seconds"]))


def main_uniform(args, taco, torch, w, plan, dev):
    paths = [p for p in (args.paths.split(",") if args.paths else plan["paths"]) if p]
    sweep_pts = plan["sweep"]
    if args.alpha is not None:
        sweep_pts = [(a, b) for a, b in sweep_pts if a == args.alpha]
    if args.beta is not None:
        sweep_pts = [(a, b) for a, b in sweep_pts if b == args.beta]
    t0 = time.time()
    X, Q = synthdata.base_and_queries(w)
    log(f"generated {w.n}x{w.d} base and {w.nq} queries in {time.time() - t0:.1f}s")
    path, oracle_build_s = cpu_baseline_index(w, X)
    S = min(args.recall_sample, w.nq)
    t0 = time.time()
    gt = ground_truth(X, Q[:S], (w.k,), dev)
    gt["n"] = S
    log(f"FP64 k-th neighbour distances of {S} queries in {time.time() - t0:.1f}s")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copied 1 GiB device-to-device for counter calibration")
    qd = torch.from_numpy(Q).to(dev)
    ids = torch.empty((w.nq, w.k), dtype=torch.int64, device=dev)
    dists = torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    tune_cache = args.tune_cache or os.path.join(os.environ.get("TMPDIR", "/tmp"), "taco_bench_tune.jsonl")

    results = {}
    for pname in paths:
        idx = taco.Index(path, 0)
        configure_path(taco, torch, idx, pname, dev, w.nq)
        tuned_cfg = None
        if PATHS[pname][2]:
            # one tuning per path, at the plan's point near the target; its
            # launch configuration serves the whole sweep
            t0 = time.time()
            ta, tb = plan["tune_at"]
            rep = idx.autotune(qd, w.k, ta, tb, cache_path=tune_cache, stream=stream)
            tuned_cfg = rep.strip().splitlines()[-1] + f" (tuned at alpha={ta} beta={tb})"
            log(f"{pname}: {tuned_cfg} in {time.time() - t0:.1f}s")
        sweep = []
        for a, b in sweep_pts:
            p = run_point(
                taco, torch, idx, pname,
                lambda: idx.search(qd, w.k, a, b, ids=ids, dists=dists, stream=stream), stream, args, w, w.nq,
                lambda: recall_at_k(ids[:S].cpu().numpy(), gt[w.k], X, Q[:S], w.k),
                lambda prec: algorithmic_bytes(idx, qd, w, a, b, prec), tuned_cfg, b, w.k)
            p.update(alpha=a, beta=b, steps=args.steps)
            sweep.append(p)
            log(f"a={a} b={b} " + describe(pname, p) +
                (f"; graph {p['graph_qps']:,.0f} QPS" if "graph_qps" in p else "") + f" [{p['seconds']:.1f}s]")
        idx.close()
        results[pname] = sweep

    main_path = plan["main"] if plan["main"] in results else paths[-1]
    sweep = results[main_path]
    value = qps_at_recall(sweep)
    op = operating_point(sweep)
    roofline = roofline_of(w.name, op, main_path)
    fp32_value = qps_at_recall(results["fp32"]) if "fp32" in results else None

    sclinear = None
    if not args.skip_sclinear:
        sclinear = sclinear_leg(taco, torch, path, qd, Q, X, gt, S, w, op, stream, args.sclinear_queries)
        sclinear["taco_qps_same_point"] = op["qps"]
        sclinear["taco_path"] = main_path
        sclinear["taco_speedup"] = op["qps"] / sclinear["qps"]
        log("SC-Linear: " + json.dumps(sclinear))

    precision = None
    if not args.skip_precision_report:
        t0 = time.time()
        pidx = taco.Index(path, 0)
        c1, c2 = index_centroids(path)
        precision = dict(cdist=cdist_errors(taco, pidx, qd, w, op["alpha"], op["beta"], c1, c2))
        if "fp32" in results:
            ref = {(p["alpha"], p["beta"]): p["recall"] for p in results["fp32"]}
            precision["recall_loss_points_vs_fp32"] = {
                pn: {f"a={p['alpha']},b={p['beta']}": 100.0 * (ref[(p["alpha"], p["beta"])] - p["recall"])
                     for p in sw if (p["alpha"], p["beta"]) in ref}
                for pn, sw in results.items() if pn != "fp32"}
        precision["bf16_rerank_recheck_fraction"] = recheck_fraction(taco, pidx, qd, w, op["alpha"], op["beta"])
        pidx.close()
        log(f"precision report in {time.time() - t0:.1f}s: " + json.dumps(precision))

    build = None
    if not args.skip_build:
        t0 = time.time()
        build = gpu_build_leg(taco, torch, w, X, dev, args.build_reps)
        obs = oracle_build_s
        if obs is None and not args.skip_cpu_baseline:
            obs = cpu_baseline_build_time(w, X)
        build["oracle_s"] = obs
        if obs:
            build["gpu_vs_oracle"] = obs * 1e3 / build["gpu_ms"]
        log(f"GPU index build: {build['gpu_ms']:.1f} ms (" + ", ".join(
            f"{k} {v:.2f}" for k, v in build["stages_ms"].items()) + f") in {time.time() - t0:.1f}s")

    cpu = None
    if not args.skip_cpu_baseline:
        cpu = cpu_baseline_leg(path, X, Q, w, gt, plan, args)

    dtype = dict(fp8="fp8+bf16", fp8_fixed="fp8+bf16", bf16="bf16", fp32="f32",
                 fp32_tuned="f32").get(main_path, "f32")
    if main_path == "tuned":
        dtype = {"bf16": "bf16+f32", "u8": "u8+f32"}.get(op.get("rerank_precision"), "f32")
    line = dict(
        metric=METRIC, value=value, unit="queries/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=op["ms_per_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype=dtype, data="synthetic",
        config=dict(workload=w.name, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l, queries_per_step=w.nq, k=w.k,
                    sweep=[list(x) for x in sweep_pts], path=main_path, alpha=op["alpha"], beta=op["beta"],
                    recall_at_10=op["recall"], recall_sample=S, batches_per_step=op["batches_per_step"],
                    tuned_config=op.get("config")),
        fp32_plain=dict(value=fp32_value, note="default options (split counting, FP32 centroid distances "
                                               "and re-rank), eager launches, default batch size"),
        speedup_vs_fp32_plain=None if not (value and fp32_value) else value / fp32_value,
        paths={pn: dict(value=qps_at_recall(sw), points=[strip_point(p) for p in sw])
               for pn, sw in results.items()},
        roofline=roofline, cpu_baseline=cpu, precision=precision, index_build=build, sclinear=sclinear)
    return line


def main_batched(args, taco, torch, w, plan, dev):
    """Per-query budgets in one tc_search_batched call per step (the batched
    configuration) against the FP32 plain path and per-query launches."""
    k_max = 100
    paths = [p for p in (args.paths.split(",") if args.paths else plan["paths"]) if p]
    betas = plan["betas"] if args.beta is None else (args.beta,)
    t0 = time.time()
    X, Q = synthdata.base_and_queries(w)
    alpha_q, k_q = synthdata.query_budgets(w.nq, w.seed)
    log(f"generated {w.n}x{w.d} base and {w.nq} queries in {time.time() - t0:.1f}s")
    path, oracle_build_s = cpu_baseline_index(w, X)
    S = min(args.recall_sample, w.nq)
    t0 = time.time()
    gt = ground_truth(X, Q[:S], (1, 10), dev)
    gt["n"] = S
    log(f"FP64 1st and 10th neighbour distances of {S} queries in {time.time() - t0:.1f}s")
    qd = torch.from_numpy(Q).to(dev)
    ad = torch.from_numpy(alpha_q).to(dev)
    kd = torch.from_numpy(k_q).to(dev)
    ids = torch.empty((w.nq, k_max), dtype=torch.int64, device=dev)
    dists = torch.empty((w.nq, k_max), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    tune_cache = args.tune_cache or os.path.join(os.environ.get("TMPDIR", "/tmp"), "taco_bench_tune.jsonl")
    rec_fn = lambda: recall_of(ids[:S].cpu().numpy(), gt, X, Q[:S], 10, k_q[:S])  # noqa: E731

    results = {}
    for pname in paths:
        idx = taco.Index(path, 0)
        tuned_cfg = None
        if pname == "batched":
            free, _ = torch.cuda.mem_get_info(dev)
            idx.set_option(taco.TC_OPT_SCRATCH_BYTES, int(free * 0.6))
            idx.set_option(taco.TC_OPT_MAX_BATCH, w.nq)
            t0 = time.time()
            tb = plan["tune_beta"]
            rep = idx.autotune_batched(qd, ad, kd, k_max, tb, cache_path=tune_cache, stream=stream)
            tuned_cfg = rep.strip().splitlines()[-1] + f" (tuned at beta={tb})"
            log(f"{pname}: {tuned_cfg} in {time.time() - t0:.1f}s")
        sweep = []
        for b in betas:
            p = run_point(
                taco, torch, idx, pname,
                lambda: idx.search_batched(qd, ad, kd, k_max, b, ids=ids, dists=dists, stream=stream),
                stream, args, w, w.nq, rec_fn,
                lambda prec: algorithmic_bytes(idx, qd, w, None, b, prec, ad, kd, k_max), tuned_cfg, b, k_max)
            p.update(alpha=None, beta=b, steps=args.steps)
            sweep.append(p)
            log(f"b={b} " + describe(pname, p) +
                (f"; graph {p['graph_qps']:,.0f} QPS ({p.get('config')})" if "graph_qps" in p else ""))
        idx.close()
        results[pname] = sweep

    # per-query launches: one tc_search call per query with its own alpha
    # and k, on a sample of the queries
    per_query = []
    m = min(plan["per_query_sample"], w.nq)
    idx = taco.Index(path, 0)
    for b in betas:
        pq_ids = torch.full((m, k_max), -1, dtype=torch.int64, device=dev)
        pq_d = torch.empty((m, k_max), dtype=torch.float32, device=dev)

        def run_pq():
            for i in range(m):
                kk = int(k_q[i])
                idx.search(qd[i:i + 1], kk, float(alpha_q[i]), b, ids=pq_ids[i:i + 1, :kk],
                           dists=pq_d[i:i + 1, :kk], stream=stream)
        run_pq()
        torch.cuda.synchronize()
        t = time.time()
        run_pq()
        torch.cuda.synchronize()
        dt = time.time() - t
        Sm = min(S, m)
        rec = recall_of(pq_ids[:Sm].cpu().numpy(), dict((k, v[:Sm]) for k, v in gt.items() if k != "n"),
                        X, Q[:Sm], 10, k_q[:Sm])
        per_query.append(dict(beta=b, qps=m / dt, recall=rec, sample=m))
        log(f"b={b} per-query launches: {m / dt:,.0f} QPS over {m} queries, recall {rec:.4f}")
    idx.close()

    main_path = plan["main"] if plan["main"] in results else paths[-1]
    sweep = results[main_path]
    op = operating_point(sweep)
    value = qps_at_recall(sweep)
    roofline = roofline_of(w.name, op, main_path)
    fp32_value = qps_at_recall(results["fp32"]) if "fp32" in results else None
    cpu = None
    if not args.skip_cpu_baseline:
        cpu = cpu_baseline_leg(path, X, Q, w, gt, plan, args, alpha_q, k_q)
    line = dict(
        metric=METRIC, value=value, unit="queries/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=op["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"bf16": "bf16+f32", "u8": "u8+f32"}.get(op.get("rerank_precision"), "f32"), data="synthetic",
        config=dict(workload=w.name, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l, queries_per_step=w.nq,
                    k="per query in {1, 10, 100}", k_max=k_max,
                    alpha="per query, log-uniform in [0.005, 0.1]", betas=list(betas), path=main_path,
                    beta=op["beta"], recall=op["recall"],
                    recall_definition="recall@10 over queries with k >= 10, recall@1 over k = 1, "
                                      "averaged by query",
                    recall_sample=S, batches_per_step=op["batches_per_step"], tuned_config=op.get("config")),
        fp32_plain=dict(value=fp32_value, note="tc_search_batched with default options, eager"),
        speedup_vs_fp32_plain=None if not (value and fp32_value) else value / fp32_value,
        per_query_launches=dict(points=per_query, value=qps_at_recall(per_query),
                                note="one tc_search call per query (its own alpha and k), default "
                                     "options, on the first queries"),
        paths={pn: dict(value=qps_at_recall(sw), points=[strip_point(p) for p in sw])
               for pn, sw in results.items()},
        roofline=roofline, cpu_baseline=cpu)
    return line


# ---------------------------------------------------------------------------
# rocprofv3 summaries (run after a profiled bench; they read only its output)
# ---------------------------------------------------------------------------

_SHORT = (("k_count_select", "count_select"), ("k_count_codes", "count_codes"), ("k_cell_bitmap", "cell_bitmap"),
          ("k_build_codes", "build_codes"), ("k_cost_order", "cost_order"), ("k_sub_dist", "sub_dist"),
          ("k_sub_select", "sub_select"), ("k_sub_count", "sub_count"), ("k_list_select", "list_select"), ("k_select_level", "select_level"), ("k_select", "select"),
          ("k_rerank16", "rerank"), ("k_rerank8", "rerank"), ("k_rerank", "rerank"),
          ("k_recheck_topk", "recheck"), ("k_stream_topk", "stream"), ("k_topk_queued", "stream"),
          ("k_topk", "topk"), ("k_probe", "probe"),
          ("k_transform", "transform"), ("k_cdist_mfma", "cdist"), ("k_qstats", "cdist"),
          ("k_prep_cent", "prep_cent"), ("k_prep_bf16", "prep_bf16"), ("k_prep_u8", "prep_u8"), ("k_qbytes", "qbytes"),
          ("k_query_order", "query_order"), ("k_flatten_cells", "flatten"),
          ("k_encode_ids", "encode_ids"), ("k_build_off2d", "build_off2d"), ("k_budgets", "budgets"),
          ("k_fill_u32", "fill"), ("k_u32_to_i64", "u32_to_i64"))


def short_kernel_name(full):
    """Short name of a library kernel (None for others).  The count kernel's
    third template argument is its form: 2 is the recount of the queries a
    list selection queued, timed within the selection stage."""
    if "taco::k_count<" in full:
        args = full.split("taco::k_count<", 1)[1].split(">", 1)[0].split(",")
        return "recount" if len(args) >= 3 and args[2].strip() == "2" else "count"
    for key, short in _SHORT:
        if "taco::" + key + "<" in full or "taco::" + key + "(" in full:
            return short
    if "taco::bld::" in full:
        # index-build kernels: build_<name without the k_ prefix>
        rest = full.split("taco::bld::", 1)[1].replace("(anonymous namespace)::", "")
        name = rest.split("(", 1)[0].split("<", 1)[0].split("::")[-1]
        return "build_" + (name[2:] if name.startswith("k_") else name)
    return None


def summarize_stats(stats_csv, bench_json, out_md, command):
    """Markdown table of rocprofv3's per-kernel statistics (its
    kernel_stats.csv, or the results database) next to the bench's own
    HIP-event timing of the same run."""
    import csv
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    if "roofline" not in line:
        return summarize_build_stats(stats_csv, line, out_md, command)
    op = line["roofline"]
    pts = line["paths"][op["path"]]["points"]
    ev = next(p for p in pts if p.get("alpha") == op.get("alpha") and p.get("beta") == op.get("beta"))["kernels"]
    if stats_csv.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(stats_csv)
        rows = [dict(Name=r[0], Calls=r[1], TotalDurationNs=r[2] * 1e3, AverageNs=r[3] * 1e3, Percentage=r[4])
                for r in con.execute("select name, total_calls, total_duration, average, percentage "
                                     "from top_kernels order by total_duration desc")]
    else:
        rows = list(csv.DictReader(open(stats_csv)))
    # per-dispatch durations (the kernel_trace.csv beside kernel_stats.csv):
    # each library kernel's launches of its largest grid, the full batches
    # the timed steps run (the other launches are sample batches)
    full = {}
    trace = stats_csv.replace("kernel_stats.csv", "kernel_trace.csv")
    if trace != stats_csv and os.path.exists(trace):
        per = {}
        for r in csv.DictReader(open(trace)):
            short = short_kernel_name(r["Kernel_Name"])
            if not short:
                continue
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            per.setdefault((r["Kernel_Name"], short), {}).setdefault(grid, []).append(dur)
        for (name, short), by_grid in per.items():
            g = max(by_grid)
            v = by_grid[g]
            full[name] = (len(v), sum(v) / len(v))
    out = [f"# rocprofv3 kernel statistics: {line['config']['workload']}, alpha={op.get('alpha')}, "
           f"beta={op.get('beta')}, {op['path']} path", "", "Command (from the repository root, TMPDIR=/tmp):", "",
           "```", command, "```", "",
           f"Tuned configuration: {line['config'].get('tuned_config')}", "",
           "The first rocprofv3 columns cover every launch of the process (warm-up, the "
           "timed steps of every sweep point, graph replays, the sample batches of the "
           "stage-count and error passes); the full-batch columns take, from the per-dispatch "
           "trace, each kernel's launches at its largest grid, i.e. the full batches of the "
           "steps; the bench column is the HIP-event average over the eager timed steps of the "
           "operating point.", "",
           "| kernel | calls | rocprof avg (us) | full-batch calls | full-batch avg (us) | bench avg (us) "
           "| rocprof total (ms) | % |",
           "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        short = short_kernel_name(r["Name"])
        b = ev.get(short, {}).get("ms_per_launch") if short else None
        fc, fa = full.get(r["Name"], (None, None))
        out.append(f"| {short or r['Name'][:40]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{'' if fc is None else fc} | {'' if fa is None else f'{fa:.1f}'} | "
                   f"{'' if b is None else f'{b * 1e3:.1f}'} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['Percentage']):.1f} |")
    if any(short_kernel_name(r["Name"]) in ("list_select", "recount") for r in rows):
        out += ["", "With the list selection, the bench's select time covers its three launches "
                "(list_select, recount and the streaming select of the queued queries); the "
                "recount is the count kernel's third form."]
    out += ["", f"Dominant kernel at the operating point: {op['kernel']}, "
            f"{op['alg_bytes_per_launch'] / 1e6:.1f} MB algorithmic per launch, "
            f"{op['achieved']:.1f} GB/s achieved = {op['frac']:.4f} of {op['peak']:.0f} GB/s.", ""]
    open(out_md, "w").write("\n".join(out))


def summarize_build_stats(stats_csv, line, out_md, command):
    """Markdown table of rocprofv3's per-kernel statistics of a --build-only
    run, with the bench's per-stage HIP-event times of the same run."""
    import csv
    b = line["index_build"]
    rows = list(csv.DictReader(open(stats_csv)))
    out = [f"# rocprofv3 kernel statistics: GPU index build (Alg 1-3), {b['workload']}", "",
           "Command (from the repository root, TMPDIR=/tmp):", "", "```", command, "```", "",
           f"n = {b['n']}, d = {b['d']}, Ns = {b['Ns']}, s = {b['s']}, l = {b['l']}, "
           f"{b['kmeans_iters']} k-means iterations; {b['reps'] + 1} builds in the process "
           "(one warm-up), so per-build counts are calls / "
           f"{b['reps'] + 1}.", "",
           "Bench stage times of the fastest build (HIP events, ms): " +
           ", ".join(f"{k} {v:.2f}" for k, v in b["stages_ms"].items()) +
           f"; total {b['gpu_ms']:.1f} ms.", "",
           "| kernel | calls | rocprof avg (us) | rocprof total (ms) | % |", "|---|---|---|---|---|"]
    for r in rows:
        short = short_kernel_name(r["Name"])
        out.append(f"| {short or r['Name'][:40]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    out += ["", "transform and encode_ids/build_off2d here are the base transform of the build and "
            "the search preparation of each built index.  The stage times above come from this "
            "profiled run: rocprofv3 adds a few microseconds to every launch, which shows in the "
            "stage made of many short launches (the one-sided eigensolver, one launch per step); "
            "the unprofiled bench line (index_build) has the plain figures.", ""]
    open(out_md, "w").write("\n".join(out))


def _counter_means(csv_path, counter):
    """Per library kernel, the mean of `counter` over its dispatches at its
    largest grid (the full batches of the timed steps; sample batches run
    smaller grids), and every copy dispatch's value."""
    import csv
    per = {}
    copies = []
    if csv_path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(csv_path)
        src = [dict(Kernel_Name=r[0], Counter_Name=r[1], Counter_Value=r[2], Grid_Size=0) for r in
               con.execute("select kernel_name, counter_name, value from counters_collection")]
    else:
        src = csv.DictReader(open(csv_path))
    for r in src:
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if "copyBuffer" in r["Kernel_Name"]:
            copies.append(v)
            continue
        short = short_kernel_name(r["Kernel_Name"])
        if short:
            per.setdefault(short, {}).setdefault(int(r.get("Grid_Size") or 0), []).append(v)
    out = {}
    for k, by_grid in per.items():
        v = by_grid[max(by_grid)]
        out[k] = (sum(v) / len(v), len(v))
    return out, copies


def summarize_traffic(fetch_csv, write_csv, bench_json, out_json, command, copy_bytes=1 << 30):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for a device copy
    of `copy_bytes` (the largest copy dispatch of the run)."""
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    fetch, fc = _counter_means(fetch_csv, "FETCH_SIZE")
    write, wc = _counter_means(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (max(fc) * 1024.0) if fc else 1.0
    w_scale = copy_bytes / (max(wc) * 1024.0) if wc else 1.0
    kern = {}
    for k in sorted(set(fetch) | set(write)):
        fk, nf = fetch.get(k, (0.0, 0))
        wk, nw = write.get(k, (0.0, 0))
        kern[k] = dict(fetch_KiB=fk, write_KiB=wk, dispatches=max(nf, nw),
                       hbm_bytes_per_launch=fk * 1024.0 * f_scale + wk * 1024.0 * w_scale)
    rec = dict(workload=line["config"]["workload"], alpha=line["config"].get("alpha"),
               beta=line["config"].get("beta"),
               path=line["config"]["path"], tuned_config=line["config"].get("tuned_config"),
               source_hash=source_hash(), copy_bytes=copy_bytes,
               fetch_scale=f_scale, write_scale=w_scale,
               copy_fetch_KiB=max(fc) if fc else None, copy_write_KiB=max(wc) if wc else None,
               command=command, kernels=kern)
    # one record per launch configuration: a summary of another
    # configuration on the same sources is kept beside this one
    keep = [r for r in traffic_records(out_json)
            if r.get("workload") == rec["workload"] and r.get("source_hash") == rec["source_hash"]
            and launch_config(r.get("tuned_config")) != launch_config(rec["tuned_config"])]
    json.dump(dict(workload=rec["workload"], records=keep + [rec]), open(out_json, "w"), indent=1)


def summarize_counters(csv_paths, out_md, command):
    """Markdown table of rocprofv3 --pmc counters per library kernel: the
    mean over its full-batch dispatches (largest grid), with the derived
    shares a 256-CU, 8-XCD MI355X gives them (GRBM_GUI_ACTIVE and the SQ
    counters are summed over the XCDs)."""
    import csv
    per = {}
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            short = short_kernel_name(r["Kernel_Name"])
            if not short:
                continue
            key = (short, r["Kernel_Name"].split("(")[0].replace("void ", "")[:48])
            per.setdefault(key, {}).setdefault(int(r["Grid_Size"]), {}).setdefault(
                r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for bg in per.values() for g in bg.values() for c in g})
    out = ["# rocprofv3 counters per kernel (full-batch dispatches)", "",
           "Commands (from the repository root, TMPDIR=/tmp):", "", "```", command, "```", "",
           "Means over each kernel's dispatches at its largest grid.  Derived: cycles = "
           "GRBM_GUI_ACTIVE / 8 (per XCD); VALU issue = SQ_INSTS_VALU / (256 CUs x cycles), one "
           "wave64 VALU instruction per cycle per CU being the peak; waits = SQ_WAIT_INST_ANY / "
           "SQ_WAVE_CYCLES; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / SQ_BUSY_CU_CYCLES.", "",
           "| kernel | dispatches | " + " | ".join(counters) + " | VALU issue | waits | MFMA busy |",
           "|---|---|" + "---|" * (len(counters) + 3)]
    for (short, name), bg in sorted(per.items(), key=lambda kv: -max(
            v[0] if v else 0 for v in [kv[1][max(kv[1])].get("GRBM_GUI_ACTIVE", [0])])):
        g = bg[max(bg)]
        m = {c: sum(v) / len(v) for c, v in g.items()}
        n = max(len(v) for v in g.values())
        cyc = m.get("GRBM_GUI_ACTIVE", 0) / 8
        valu = f"{m['SQ_INSTS_VALU'] / (256 * cyc):.2f}" if cyc and "SQ_INSTS_VALU" in m else ""
        wait = (f"{m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.2f}"
                if m.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_ANY" in m else "")
        mf = (f"{m['SQ_VALU_MFMA_BUSY_CYCLES'] / m['SQ_BUSY_CU_CYCLES']:.4f}"
              if m.get("SQ_BUSY_CU_CYCLES") and "SQ_VALU_MFMA_BUSY_CYCLES" in m else "")
        out.append(f"| {short} ({name}) | {n} | " + " | ".join(
            f"{m[c]:.4g}" if c in m else "" for c in counters) + f" | {valu} | {wait} | {mf} |")
    open(out_md, "w").write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(PLANS))
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None, help="run only the sweep points with this alpha")
    ap.add_argument("--beta", type=float, default=None, help="run only the sweep points with this beta")
    ap.add_argument("--paths", default=None,
                    help="comma list of paths (default: the workload's plan): fp32, fp32_tuned, "
                         "tuned, bf16, fp8, fp8_fixed (the fixed-budget selection); batched for "
                         "zipf-1m-d256")
    ap.add_argument("--skip-precision-report", action="store_true")
    ap.add_argument("--skip-build", action="store_true", help="omit the GPU index-build leg")
    ap.add_argument("--skip-sclinear", action="store_true", help="omit the SC-Linear leg")
    ap.add_argument("--sclinear-queries", type=int, default=1000)
    ap.add_argument("--build-only", action="store_true",
                    help="run only the GPU index-build leg (and the oracle's build time unless "
                         "--skip-cpu-baseline); prints its own JSON line")
    ap.add_argument("--build-reps", type=int, default=3)
    ap.add_argument("--skip-cpu-baseline", action="store_true",
                    help="omit the oracle timing (profiling runs); the line then has no cpu_baseline")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file (JSON lines); default a file under TMPDIR")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a known-size kernel for counter scaling)")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("KERNEL_STATS_CSV", "BENCH_JSON"))
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"))
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_CSV")
    ap.add_argument("--summary-out")
    ap.add_argument("--summary-command", default="")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, args.summary_out, args.summary_command)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.summary_out, args.summary_command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.summary_out, args.summary_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps(dict(error="the benchmark runs on one GPU only: the path is measured on one GPU's "
                                    "share; run with --gpus 1", n_gpus=args.gpus)), flush=True)
        sys.exit(2)

    import torch
    import paper_2603_24919_amd as taco

    w = synthdata.WORKLOADS[args.workload]
    plan = PLANS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.build_only:
        t0 = time.time()
        X, _ = synthdata.base_and_queries(w, nq=0)
        log(f"generated {w.n}x{w.d} base in {time.time() - t0:.1f}s")
        build = gpu_build_leg(taco, torch, w, X, dev, args.build_reps)
        if not args.skip_cpu_baseline:
            build["oracle_s"] = cpu_baseline_build_time(w, X)
            build["gpu_vs_oracle"] = build["oracle_s"] * 1e3 / build["gpu_ms"]
        log(f"GPU index build: {build['gpu_ms']:.1f} ms (" + ", ".join(
            f"{k} {v:.2f}" for k, v in build["stages_ms"].items()) + ")")
        print(json.dumps(dict(metric="GPU index build time (Alg 1-3)", value=build["gpu_ms"], unit="ms",
                              n_gpus=1, higher_is_better=False, data="synthetic",
                              config=dict(workload=w.name), index_build=build)), flush=True)
        return
    line = main_batched(args, taco, torch, w, plan, dev) if "betas" in plan else \
        main_uniform(args, taco, torch, w, plan, dev)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
