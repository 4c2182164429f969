"""Throughput of the TaCo query stage on one MI355X.

One step = one pass of the whole query path (transform, probe, collision
count, candidate selection, re-rank, top-k) over one batch of queries that is
already resident in HBM.  The workload is the 1M x 128 integer Gaussian
mixture (1,024 components, sigma U[5,25]) with Ns=8 subspaces of 16 dims,
50x50 IMI cells per subspace, 10,000 queries, k=10, beta=0.005, swept over
alpha in {0.01, 0.03, 0.05}.  The reported value is QPS at recall@10 = 0.95,
read off the (recall, QPS) points of the sweep (recall from FP64 ground
truth on a sample of the queries).

Legs:
  * cpu_baseline leg (the oracle, test infrastructure): builds the serialized
    index from the workload's seed (the index builder of the method is the
    oracle's Alg 1-3), computes the FP64 ground truth of the recall sample,
    and times the oracle's own query on a bounded sample on the host cores.
  * GPU leg: loads the index through the C-ABI and times K steps per alpha
    with HIP events on the search stream, per kernel as well.

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
KERNELS = ("transform", "probe", "count", "select", "rerank", "topk")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# cpu_baseline leg: everything that runs the oracle lives here
# ---------------------------------------------------------------------------

def cpu_baseline_index(w, X):
    """Serialized index built by the oracle from the workload seed (cached)."""
    from oracle import oracle as O
    cache = os.environ.get("TACO_CACHE") or os.path.join(ROOT, ".taco_cache")
    os.makedirs(cache, exist_ok=True)
    path = os.path.join(cache, f"{w.name}-n{w.n}-s{w.seed:x}.tcx")
    if not os.path.exists(path):
        t = time.time()
        tmp = path + ".tmp%d" % os.getpid()
        O.build_workload_index(w, tmp, X)
        os.replace(tmp, path)
        log(f"oracle built the index in {time.time() - t:.1f}s -> {path}")
    return path


def cpu_baseline_ground_truth(X, Qs, k):
    from oracle import oracle as O
    t = time.time()
    ids, d64 = O.bruteforce(X, Qs, k)
    log(f"FP64 ground truth for {Qs.shape[0]} queries in {time.time() - t:.1f}s")
    return ids, d64


def cpu_baseline_recall(ids, gt_d64, X, Qs, k):
    from oracle import oracle as O
    return O.recall_at_k(ids, gt_d64, X, Qs, k)


def cpu_baseline_timing(path, X, Q, w, gt, alphas, sample):
    """The oracle as it stands, parallel over queries with OpenMP on the host
    cores, on `sample` queries per alpha; one warm-up query first."""
    from oracle import oracle as O
    oidx = O.OracleIndex(path)
    threads = O.max_threads()
    pts = []
    Qs = Q[:sample]
    for a in alphas:
        oidx.query_batch(Qs[:threads], a, w.beta, w.k)
        t = time.time()
        ids = oidx.query_batch(Qs, a, w.beta, w.k)
        dt = time.time() - t
        rec = O.recall_at_k(ids, gt[1][:sample], X, Qs, w.k)
        pts.append(dict(alpha=a, qps=sample / dt, recall=rec, seconds=dt))
        log(f"oracle alpha={a}: {sample / dt:.1f} QPS on {threads} threads, recall {rec:.4f}")
    oidx.close()
    return pts, threads


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def qps_at_recall(points, target=RECALL_TARGET):
    """QPS at the target recall from (recall, qps) points: the best QPS of a
    point at or above the target, or the linear interpolation between a
    faster point below and a slower point above it (Pareto frontier)."""
    best = None
    for p in points:
        if p["recall"] >= target:
            best = p["qps"] if best is None else max(best, p["qps"])
    for lo in points:
        for hi in points:
            if lo["recall"] < target <= hi["recall"] and lo["qps"] > hi["qps"]:
                f = (hi["recall"] - target) / (hi["recall"] - lo["recall"])
                v = hi["qps"] + f * (lo["qps"] - hi["qps"])
                best = v if best is None else max(best, v)
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


def algorithmic_bytes(idx, q, w, alpha, nq):
    """Bytes the method must move, per kernel, for one step at this alpha:
    count: ids of the probed lists (4 B each) + the slice bounds and probed
    cell ids (12 B per probed cell); select: the candidate ids written (4 B);
    rerank: each candidate's row (4d B), id and distance (8 B) plus the query
    (4d B); topk: candidate keys (8 B each) and the output (12k B)."""
    import torch
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
        rerank=C * (4.0 * d + 8.0) + nq * 4.0 * d,
        topk=8.0 * C + 12.0 * w.k * nq,
    ), dict(retrieved=R / nq, probed_cells=P / nq, candidates=C / nq)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=400)
    ap.add_argument("--skip-cpu-baseline", action="store_true",
                    help="omit the oracle timing (profiling runs); the line then has no cpu_baseline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps(dict(error="this build measures one GPU only; run with --gpus 1",
                              n_gpus=args.gpus)), flush=True)
        sys.exit(2)

    import torch
    import paper_2603_24919_amd as taco

    w = synthdata.WORKLOADS[WORKLOAD]
    t0 = time.time()
    X, Q = synthdata.base_and_queries(w)
    log(f"generated {w.n}x{w.d} base and {w.nq} queries in {time.time() - t0:.1f}s")
    path = cpu_baseline_index(w, X)
    S = min(args.recall_sample, w.nq)
    gt = cpu_baseline_ground_truth(X, Q[:S], w.k)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    idx = taco.Index(path, 0)
    qd = torch.from_numpy(Q).to(dev)
    ids = torch.empty((w.nq, w.k), dtype=torch.int64, device=dev)
    dists = torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    batches = -(-w.nq // idx.batch_capacity())

    sweep = []
    for a in w.alphas:
        for _ in range(args.warmup):
            idx.search(qd, w.k, a, w.beta, ids=ids, dists=dists, stream=stream)
        torch.cuda.synchronize()
        idx.set_option(taco.TC_OPT_PROFILE, 1)
        idx.profile_reset()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            idx.search(qd, w.k, a, w.beta, ids=ids, dists=dists, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        kern = {}
        for kname in KERNELS:
            tot, n = idx.kernel_time(kname)
            kern[kname] = dict(ms_total=tot, launches=n)
        idx.set_option(taco.TC_OPT_PROFILE, 0)
        rec = cpu_baseline_recall(ids[:S].cpu().numpy(), gt[1], X, Q[:S], w.k)
        alg, avg = algorithmic_bytes(idx, qd, w, a, w.nq)
        for kname in KERNELS:
            launches = max(kern[kname]["launches"], 1)
            kern[kname]["ms_per_launch"] = kern[kname]["ms_total"] / launches
            kern[kname]["alg_bytes_per_launch"] = alg[kname] / batches
            kern[kname]["alg_GBps"] = (alg[kname] / batches) / (kern[kname]["ms_per_launch"] * 1e-3) / 1e9 \
                if kern[kname]["ms_per_launch"] > 0 else None
        qps = w.nq * args.steps / (ms * 1e-3)
        sweep.append(dict(alpha=a, qps=qps, recall=rec, ms_per_step=ms / args.steps, kernels=kern,
                          per_query=avg))
        log(f"GPU alpha={a}: {qps:,.0f} QPS, {ms / args.steps:.3f} ms/step, recall@10 {rec:.4f}; "
            + ", ".join(f"{k} {v['ms_total'] / args.steps:.3f}" for k, v in kern.items()))

    value = qps_at_recall(sweep)
    # operating point: the fastest alpha at or above the target (else the
    # most accurate one)
    ok = [p for p in sweep if p["recall"] >= RECALL_TARGET]
    op = max(ok, key=lambda p: p["qps"]) if ok else max(sweep, key=lambda p: p["recall"])
    dom = max(KERNELS, key=lambda k_: op["kernels"][k_]["ms_total"])
    dk = op["kernels"][dom]
    achieved = dk["alg_GBps"]
    traffic = traffic_from_profiles(dom)
    roofline = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=None if achieved is None else achieved / HBM_PEAK_GBS,
                    traffic=traffic, alg_bytes_per_launch=dk["alg_bytes_per_launch"],
                    ms_per_launch=dk["ms_per_launch"])

    cpu = None
    if not args.skip_cpu_baseline:
        pts, threads = cpu_baseline_timing(path, X, Q, w, gt, w.alphas, min(args.cpu_sample, S))
        cpu_v = qps_at_recall(pts)
        cpu = dict(value=cpu_v, unit="queries/s", cores=threads, kind="oracle",
                   sample=f"first {min(args.cpu_sample, S)} queries at each alpha of the sweep, "
                          f"OpenMP over queries; value read at recall@10=0.95 like the GPU's",
                   points=[dict(alpha=p["alpha"], qps=p["qps"], recall=p["recall"]) for p in pts])

    line = dict(
        metric=METRIC, value=value, unit="queries/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=op["ms_per_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD, n=w.n, d=w.d, Ns=w.Ns, s=w.s, l=w.l,
                    queries_per_step=w.nq, k=w.k, beta=w.beta, alphas=list(w.alphas),
                    alpha=op["alpha"], path="fp32-plain", recall_at_10=op["recall"],
                    recall_sample=S, batches_per_step=batches),
        sweep=[dict(alpha=p["alpha"], qps=p["qps"], recall=p["recall"], ms_per_step=p["ms_per_step"],
                    per_query=p["per_query"],
                    kernels={k_: dict(ms_per_launch=v["ms_per_launch"], launches=v["launches"],
                                      alg_GBps=v["alg_GBps"]) for k_, v in p["kernels"].items()})
               for p in sweep],
        roofline=roofline, cpu_baseline=cpu)
    idx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
