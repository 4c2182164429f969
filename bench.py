"""Throughput of the TaCo query stage on one MI355X.

One step = one pass of the whole query path (transform, probe, collision
count, candidate selection, re-rank, top-k) over one batch of queries that is
already resident in HBM.  The workload is the 1M x 128 integer Gaussian
mixture (1,024 components, sigma U[5,25]) with Ns=8 subspaces of 16 dims,
50x50 IMI cells per subspace, 10,000 queries, k=10, beta=0.005, swept over
alpha in {0.01, 0.03, 0.05}.  The reported value is QPS at recall@10 = 0.95,
read off the Pareto frontier of the (recall, QPS) points of the sweep;
recall is tie-aware against FP64 exact k-NN distances of a sample of the
queries (computed here with numpy).

Legs:
  * cpu_baseline leg (the oracle, test infrastructure): builds the serialized
    index from the workload's seed (the index builder of the method is the
    oracle's Alg 1-3; both paths search this same file) and times the
    oracle's own query on a bounded sample on the host cores.
  * GPU leg: loads the index through the C-ABI and times K steps per alpha
    with HIP events on the search stream, per kernel as well, on three
    paths: "fp32" (default launch configuration, FP32 re-rank), "tuned" (the
    library's autotuner picks tile width, count mode, probe packing, re-rank
    spread and re-rank precision per alpha; results are identical to FP32)
    and "lowp" (tuned, plus FP8 centroid distances on the matrix cores,
    which may change the probe near ties).  Tuned and lowp run as captured
    HIP graphs (TC_OPT_GRAPH): their QPS is the replay rate, with recall read
    from the replays' results, and an eager run gives the per-kernel timing
    (eager_qps beside it).  The reported value is the tuned path's; all paths
    are listed under "paths".
  * precision report: relative error of the BF16 and FP8 centroid distances
    against FP64, recall@10 of each form per alpha and its loss against the
    FP32 form, and the fraction of candidates the BF16 re-rank re-checks.

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

WORKLOAD = "gmm-int-1m-d128"
METRIC = "QPS at recall@10=0.95 on 1 MI355X; BF16/FP8+batched vs FP32 plain"
RECALL_TARGET = 0.95
HBM_PEAK_GBS = 8000.0
KERNELS = ("transform", "probe", "count", "select", "rerank", "topk", "recheck", "count_select")


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
    scratch file, removed afterwards): the index-build baseline when the
    cached index was not built in this run."""
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


BUILD_STAGES = ("stats", "eigen", "allocate", "transform", "kmeans", "imi")


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
    best = min(runs, key=lambda m: float(m.sum()))
    return dict(workload=WORKLOAD, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l, kmeans_iters=w.iters,
                gpu_ms=float(best.sum()), stages_ms=dict(zip(BUILD_STAGES, map(float, best))),
                reps=reps, timing="HIP events around each stage, base resident in HBM; the "
                                  "index's search preparation and the host copies excluded")


def cpu_baseline_timing(path, X, Q, w, kth, alphas, sample):
    """The oracle as it stands, parallel over queries with OpenMP on the host
    cores, timed on the first `sample` queries per alpha (one warm-up batch
    first); its recall is read on the first queries that have ground truth."""
    from oracle import oracle as O
    oidx = O.OracleIndex(path)
    threads = O.max_threads()
    pts = []
    Qs = Q[:sample]
    S = min(sample, kth.shape[0])
    for a in alphas:
        oidx.query_batch(Qs[:threads], a, w.beta, w.k)
        t = time.time()
        ids = oidx.query_batch(Qs, a, w.beta, w.k)
        dt = time.time() - t
        rec = recall_at_k(ids[:S], kth[:S], X, Qs[:S], w.k)
        pts.append(dict(alpha=a, qps=sample / dt, recall=rec, seconds=dt))
        log(f"oracle alpha={a}: {sample / dt:.1f} QPS on {threads} threads over {sample} queries, "
            f"recall {rec:.4f}")
    oidx.close()
    return pts, threads


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def kth_neighbour_fp64(X, Qs, k, chunk=64):
    """FP64 squared distance of each query's k-th nearest base row: a
    shortlist of k+32 rows from the expanded form |x|^2 - 2 x.q in FP64,
    then the direct sum of squared differences on the shortlist."""
    X64 = X.astype(np.float64)
    xn = (X64 * X64).sum(1)
    out = np.empty(Qs.shape[0])
    m = min(k + 32, X.shape[0])
    for c0 in range(0, Qs.shape[0], chunk):
        q = Qs[c0:c0 + chunk].astype(np.float64)
        approx = xn[None, :] - 2.0 * (q @ X64.T)
        short = np.argpartition(approx, m - 1, axis=1)[:, :m]
        for i in range(q.shape[0]):
            d = ((X64[short[i]] - q[i]) ** 2).sum(1)
            out[c0 + i] = np.sort(d)[k - 1]
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


def index_centroids(path):
    """The half-subspace centroids C1 [Ns][l][h1], C2 [Ns][l][h2] read from
    the index file (128-byte header, then mean, B, C1, C2, all f32)."""
    hdr = np.fromfile(path, dtype=np.uint8, count=128)
    d, Ns, s, h1, h2, l = (int(v) for v in hdr[24:48].view(np.int32))
    off = 128 + 4 * (d + d * Ns * s)
    c1 = np.fromfile(path, dtype=np.float32, count=Ns * l * h1, offset=off).reshape(Ns, l, h1)
    c2 = np.fromfile(path, dtype=np.float32, count=Ns * l * h2, offset=off + 4 * Ns * l * h1).reshape(Ns, l, h2)
    return c1, c2


def precision_report(taco, path, qd, w, X, Q, kth, S, alpha, nq_err=200):
    """The reduced-precision forms against FP64 and against the FP32 form:
    relative error of the centroid distances (BF16 / FP8 on the matrix
    cores), recall@10 of each form at every alpha, and for the BF16 re-rank
    the fraction of candidates re-checked in FP32."""
    import torch
    c1, c2 = index_centroids(path)
    Ns, l, h1 = c1.shape
    rep = {}
    forms = (("fp32", taco.TC_CDIST_FP32), ("bf16", taco.TC_CDIST_BF16), ("fp8", taco.TC_CDIST_FP8))
    for name, val in forms:
        idx = taco.Index(path, 0)
        idx.set_option(taco.TC_OPT_CDIST_PRECISION, val)
        P = min(nq_err, w.nq)
        dump = idx.dump_buffers(P, ("qt", "cdist"))
        idx.search_debug(qd[:P], w.k, alpha, w.beta, dump)
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
        recalls = {}
        ids = torch.empty((w.nq, w.k), dtype=torch.int64, device=qd.device)
        dists = torch.empty((w.nq, w.k), dtype=torch.float32, device=qd.device)
        for a in w.alphas:
            idx.search(qd, w.k, a, w.beta, ids=ids, dists=dists)
            torch.cuda.synchronize()
            recalls[a] = recall_at_k(ids[:S].cpu().numpy(), kth, X, Q[:S], w.k)
        idx.close()
        rep[name] = dict(cdist_rel_err_max=float(rel.max()), cdist_rel_err_mean=float(rel.mean()),
                         recall_at_10=recalls)
    for name in ("bf16", "fp8"):
        rep[name]["recall_loss_points"] = {a: 100.0 * (rep["fp32"]["recall_at_10"][a] - rep[name]["recall_at_10"][a])
                                           for a in w.alphas}
    idx = taco.Index(path, 0)
    idx.set_option(taco.TC_OPT_PRECISION, taco.TC_BF16)
    dump = idx.dump_buffers(w.nq, ("ncand", "nrecheck"))
    idx.search_debug(qd, w.k, alpha, w.beta, dump)
    torch.cuda.synchronize()
    rep["bf16_rerank_recheck_fraction"] = float(dump["nrecheck"].sum().item()) / max(1.0, float(dump["ncand"].sum().item()))
    idx.close()
    rep["cdist_error_sample"] = f"first {min(nq_err, w.nq)} queries, all half-subspace centroids, alpha={alpha}"
    return rep


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


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "runtime.cpp"):
        with open(os.path.join(ROOT, "paper_2603_24919_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    if rec.get("source_hash") != source_hash() or rec.get("workload") != WORKLOAD:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def algorithmic_bytes(idx, q, w, alpha, nq, precision=0):
    """Bytes the method must move, per kernel, for one step at this alpha:
    count: ids of the probed lists (4 B each) + the slice bounds and probed
    cell ids (12 B per probed cell); select: the candidate ids written (4 B);
    count_select: both; rerank: each candidate's row (4d B; 2d B plus its
    4 B error bound in BF16; d B plus offset, step and error bound, 12 B, in
    8 bits), id and distance (8 B) plus the query (4d B);
    topk: candidate keys (8 B each) and the output (12k B); recheck: the
    candidates' lower bounds (4 B each)."""
    import torch
    import paper_2603_24919_amd as taco
    dump = idx.dump_buffers(nq, ("retrieved", "ncells", "ncand"))
    idx.search_debug(q, w.k, alpha, w.beta, dump)
    torch.cuda.synchronize()
    R = float(dump["retrieved"].sum().item())
    P = float(dump["ncells"].sum().item())
    C = float(dump["ncand"].sum().item())
    d = w.d
    return dict(
        transform=nq * (4.0 * d + 4.0 * w.M),
        probe=nq * w.M * 4.0 + 4.0 * P,
        count=4.0 * R + 12.0 * P,
        select=4.0 * C + 4.0 * P,
        count_select=4.0 * R + 16.0 * P + 4.0 * C,
        rerank=C * ({0: 4.0 * d, 1: 2.0 * d + 4.0, 2: d + 12.0}[precision] + 8.0) + nq * 4.0 * d,
        topk=8.0 * C + 12.0 * w.k * nq,
        recheck=4.0 * C,
    ), dict(retrieved=R / nq, probed_cells=P / nq, candidates=C / nq)


# ---------------------------------------------------------------------------
# rocprofv3 summaries (run after a profiled bench; they read only its CSVs)
# ---------------------------------------------------------------------------

_SHORT = (("k_count_select", "count_select"), ("k_list_select", "list_select"), ("k_select_level", "select_level"), ("k_select", "select"),
          ("k_rerank16", "rerank"), ("k_rerank8", "rerank"), ("k_rerank", "rerank"),
          ("k_recheck_topk", "recheck"), ("k_topk", "topk"), ("k_probe", "probe"),
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
    ev = next(p for p in pts if p["alpha"] == op["alpha"])["kernels"]
    if stats_csv.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(stats_csv)
        rows = [dict(Name=r[0], Calls=r[1], TotalDurationNs=r[2] * 1e3, AverageNs=r[3] * 1e3, Percentage=r[4])
                for r in con.execute("select name, total_calls, total_duration, average, percentage "
                                     "from top_kernels order by total_duration desc")]
    else:
        rows = list(csv.DictReader(open(stats_csv)))
    out = [f"# rocprofv3 kernel statistics: {line['config']['workload']}, alpha={op['alpha']}, "
           f"{op['path']} path", "", "Command (from the repository root, TMPDIR=/tmp):", "",
           "```", command, "```", "",
           f"Tuned configuration: {line['config'].get('tuned_config')}", "",
           "rocprofv3 averages cover every launch of the process (warm-up, the timed steps, the "
           "stage-count pass and the recall pass); the bench column is the HIP-event average "
           "over the timed steps only.", "",
           "| kernel | calls | rocprof avg (us) | bench avg (us) | rocprof total (ms) | % |",
           "|---|---|---|---|---|---|"]
    for r in rows:
        short = short_kernel_name(r["Name"])
        b = ev.get(short, {}).get("ms_per_launch") if short else None
        out.append(f"| {short or r['Name'][:40]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
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
    import csv
    per = {}
    copies = []
    if csv_path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(csv_path)
        src = [dict(Kernel_Name=r[0], Counter_Name=r[1], Counter_Value=r[2]) for r in
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
            per.setdefault(short, []).append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in per.items()}, copies


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
    rec = dict(workload=line["config"]["workload"], alpha=line["config"]["alpha"],
               path=line["config"]["path"], tuned_config=line["config"].get("tuned_config"),
               source_hash=source_hash(), copy_bytes=copy_bytes,
               fetch_scale=f_scale, write_scale=w_scale,
               copy_fetch_KiB=max(fc) if fc else None, copy_write_KiB=max(wc) if wc else None,
               command=command, kernels=kern)
    json.dump(rec, open(out_json, "w"), indent=1)


def timed_steps(idx, taco, qd, w, a, ids, dists, stream, steps, warmup, profile=True):
    """Warm-up, then exactly `steps` searches of the whole batch between two
    events on the search stream.  Returns (ms, per-kernel totals)."""
    import torch
    for _ in range(warmup):
        idx.search(qd, w.k, a, w.beta, ids=ids, dists=dists, stream=stream)
    torch.cuda.synchronize()
    if profile:
        idx.set_option(taco.TC_OPT_PROFILE, 1)
        idx.profile_reset()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        idx.search(qd, w.k, a, w.beta, ids=ids, dists=dists, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    kern = {}
    if profile:
        for kname in KERNELS:
            tot, n = idx.kernel_time(kname)
            kern[kname] = dict(ms_total=tot, launches=n)
        idx.set_option(taco.TC_OPT_PROFILE, 0)
    return start.elapsed_time(stop), kern


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=4000)
    ap.add_argument("--alpha", type=float, default=None,
                    help="run only this collision ratio of the sweep (profiling runs)")
    ap.add_argument("--paths", default="fp32,fixed,tuned,lowp",
                    help="comma list of fp32 (defaults), fixed (defaults with the fixed-budget "
                         "selection rule, SuCo's, in place of Alg 5), tuned (autotuned, exact), lowp "
                         "(tuned + FP8 centroid distances on the matrix cores)")
    ap.add_argument("--skip-precision-report", action="store_true")
    ap.add_argument("--skip-build", action="store_true", help="omit the GPU index-build leg")
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
    ap.add_argument("--summary-out")
    ap.add_argument("--summary-command", default="")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, args.summary_out, args.summary_command)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.summary_out, args.summary_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps(dict(error="the benchmark runs on one GPU only: the path is measured on one GPU's share; run with --gpus 1",
                              n_gpus=args.gpus)), flush=True)
        sys.exit(2)

    import torch
    import paper_2603_24919_amd as taco

    w = synthdata.WORKLOADS[WORKLOAD]
    alphas = list(w.alphas) if args.alpha is None else [args.alpha]
    paths = [p for p in args.paths.split(",") if p]
    t0 = time.time()
    X, Q = synthdata.base_and_queries(w)
    log(f"generated {w.n}x{w.d} base and {w.nq} queries in {time.time() - t0:.1f}s")
    path, oracle_build_s = cpu_baseline_index(w, X)
    S = min(args.recall_sample, w.nq)
    t0 = time.time()
    kth = kth_neighbour_fp64(X, Q[:S], w.k)
    log(f"FP64 k-th neighbour distances of {S} queries in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.build_only:
        build = gpu_build_leg(taco, torch, w, X, dev, args.build_reps)
        obs = oracle_build_s
        if obs is None and not args.skip_cpu_baseline:
            obs = cpu_baseline_build_time(w, X)
        build["oracle_s"] = obs
        if obs:
            build["gpu_vs_oracle"] = obs * 1e3 / build["gpu_ms"]
        log(f"GPU index build: {build['gpu_ms']:.1f} ms (" + ", ".join(
            f"{k} {v:.2f}" for k, v in build["stages_ms"].items()) + ")")
        print(json.dumps(dict(metric="GPU index build time (Alg 1-3)", value=build["gpu_ms"], unit="ms",
                              n_gpus=1, higher_is_better=False, data="synthetic",
                              config=dict(workload=WORKLOAD), index_build=build)), flush=True)
        return
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
        if pname == "fixed":
            idx.set_option(taco.TC_OPT_SELECT_RULE, taco.TC_RULE_FIXED)
        if pname in ("tuned", "lowp"):
            # one batch per step when the GPU has room: candidate scratch is sized for the
            # worst case (every point a candidate), ~12.5 MB per query at 1M points, so a
            # 10k-query batch takes ~125 GB of the 288 GB; at most 60% of what is free
            free, _ = torch.cuda.mem_get_info(dev)
            idx.set_option(taco.TC_OPT_SCRATCH_BYTES, int(free * 0.6))
            idx.set_option(taco.TC_OPT_MAX_BATCH, w.nq)
        sweep = []
        for a in alphas:
            tuned = None
            if pname in ("tuned", "lowp"):
                tuned = idx.autotune(qd, w.k, a, w.beta, cache_path=tune_cache, stream=stream)
                log(f"{pname} alpha={a}: " + tuned.strip().splitlines()[-1])
            if pname == "lowp":
                idx.set_option(taco.TC_OPT_CDIST_PRECISION, taco.TC_CDIST_FP8)
            batches = -(-w.nq // idx.batch_capacity())
            ms, kern = timed_steps(idx, taco, qd, w, a, ids, dists, stream, args.steps, args.warmup)
            rec = recall_at_k(ids[:S].cpu().numpy(), kth, X, Q[:S], w.k)
            prec = 0
            if tuned is not None and "precision=" in tuned:
                prec = int(tuned.strip().splitlines()[-1].split("precision=")[1].split()[0])
            alg, avg = algorithmic_bytes(idx, qd, w, a, w.nq, precision=prec)
            for kname in KERNELS:
                launches = max(kern[kname]["launches"], 1)
                kern[kname]["ms_per_launch"] = kern[kname]["ms_total"] / launches
                b = alg.get(kname)
                kern[kname]["alg_bytes_per_launch"] = None if b is None else b * args.steps / launches
                kern[kname]["alg_GBps"] = None if (b is None or kern[kname]["ms_total"] <= 0) else \
                    (b * args.steps) / (kern[kname]["ms_total"] * 1e-3) / 1e9
            qps = w.nq * args.steps / (ms * 1e-3)
            point = dict(alpha=a, qps=qps, recall=rec, ms_per_step=ms / args.steps, kernels=kern,
                         per_query=avg, batches_per_step=batches)
            if tuned is not None:
                # the tuned paths run as the library's captured graph (TC_OPT_GRAPH): the value is
                # the replay rate, with recall re-read from the replays' own results; the eager
                # run above gives the per-kernel timing
                point["config"] = tuned.strip().splitlines()[-1] + (" cdist=fp8" if pname == "lowp" else "")
                idx.set_option(taco.TC_OPT_GRAPH, 1)
                ids.fill_(-1)
                gms, _ = timed_steps(idx, taco, qd, w, a, ids, dists, stream, args.steps, args.warmup,
                                     profile=False)
                idx.set_option(taco.TC_OPT_GRAPH, 0)
                grec = recall_at_k(ids[:S].cpu().numpy(), kth, X, Q[:S], w.k)
                point.update(eager_qps=qps, eager_ms_per_step=ms / args.steps,
                             graph_qps=w.nq * args.steps / (gms * 1e-3))
                point.update(qps=point["graph_qps"], ms_per_step=gms / args.steps, recall=min(rec, grec))
            sweep.append(point)
            log(f"{pname} alpha={a}: eager {qps:,.0f} QPS, {ms / args.steps:.3f} ms/step, recall@10 {rec:.4f}; "
                + ", ".join(f"{k} {v['ms_total'] / args.steps:.3f}" for k, v in kern.items()
                            if v["ms_total"] > 0)
                + (f"; graph {point['graph_qps']:,.0f} QPS" if "graph_qps" in point else ""))
        idx.close()
        results[pname] = sweep

    main_path = "tuned" if "tuned" in results else paths[0]
    sweep = results[main_path]
    value = qps_at_recall(sweep)
    ok = [p for p in sweep if p["recall"] >= RECALL_TARGET]
    op = max(ok, key=lambda p: p["qps"]) if ok else max(sweep, key=lambda p: p["recall"])
    dom = max(op["kernels"], key=lambda k_: op["kernels"][k_]["ms_total"])
    dk = op["kernels"][dom]
    achieved = dk["alg_GBps"]
    traffic = traffic_from_profiles(dom)
    roofline = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=None if achieved is None else achieved / HBM_PEAK_GBS,
                    traffic=traffic, alg_bytes_per_launch=dk["alg_bytes_per_launch"],
                    ms_per_launch=dk["ms_per_launch"], alpha=op["alpha"], path=main_path)

    build = None
    if not args.skip_build:
        t0 = time.time()
        build = gpu_build_leg(taco, torch, w, X, dev, args.build_reps)
        if oracle_build_s is None and not args.skip_cpu_baseline:
            oracle_build_s = cpu_baseline_build_time(w, X)
        build["oracle_s"] = oracle_build_s
        build["oracle_note"] = ("the oracle's build of the same index (Alg 1-3, OpenMP over points on the "
                                "host cores) in this run" if oracle_build_s is not None else "not timed")
        if oracle_build_s:
            build["gpu_vs_oracle"] = oracle_build_s * 1e3 / build["gpu_ms"]
        log(f"GPU index build: {build['gpu_ms']:.1f} ms (" + ", ".join(
            f"{k} {v:.2f}" for k, v in build["stages_ms"].items()) + f") in {time.time() - t0:.1f}s")

    precision = None
    if not args.skip_precision_report:
        t0 = time.time()
        precision = precision_report(taco, path, qd, w, X, Q, kth, S, op["alpha"])
        log(f"precision report in {time.time() - t0:.1f}s: " + json.dumps(precision))

    cpu = None
    if not args.skip_cpu_baseline:
        cs = min(args.cpu_sample, w.nq)
        pts, threads = cpu_baseline_timing(path, X, Q, w, kth, alphas, cs)
        cpu = dict(value=qps_at_recall(pts), unit="queries/s", cores=threads, kind="oracle",
                   sample=f"first {cs} of the {w.nq} queries at each alpha of the sweep, OpenMP over "
                          f"queries, recall on the first {min(cs, S)}; value read at recall@10=0.95 "
                          f"like the GPU's",
                   seconds=sum(p["seconds"] for p in pts),
                   points=[dict(alpha=p["alpha"], qps=p["qps"], recall=p["recall"]) for p in pts])

    cfg = str(op.get("config", ""))
    line = dict(
        metric=METRIC, value=value, unit="queries/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=op["ms_per_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None,
        dtype="bf16+f32" if "precision=1" in cfg else ("u8+f32" if "precision=2" in cfg else "f32"),
        data="synthetic",
        config=dict(workload=WORKLOAD, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l,
                    queries_per_step=w.nq, k=w.k, beta=w.beta, alphas=alphas,
                    alpha=op["alpha"], path=main_path, recall_at_10=op["recall"],
                    recall_sample=S, batches_per_step=op["batches_per_step"],
                    tuned_config=op.get("config")),
        paths={pn: dict(value=qps_at_recall(sw),
                        points=[dict(alpha=p["alpha"], qps=p["qps"], recall=p["recall"],
                                     ms_per_step=p["ms_per_step"], graph_qps=p.get("graph_qps"),
                                     eager_qps=p.get("eager_qps"),
                                     config=p.get("config"), per_query=p["per_query"],
                                     kernels={k_: dict(ms_per_launch=v["ms_per_launch"],
                                                       launches=v["launches"], alg_GBps=v["alg_GBps"])
                                              for k_, v in p["kernels"].items() if v["launches"]})
                                for p in sw])
               for pn, sw in results.items()},
        roofline=roofline, cpu_baseline=cpu, precision=precision, index_build=build)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
