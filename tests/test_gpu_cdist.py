"""Reduced-precision centroid distances (BF16 / FP8 e4m3 on the matrix cores).

This form is not the paper's; it only reorders the probe near ties.  Checks:
* every distance lies within a bound derived from the operand formats' unit
  roundoffs around the FP64 distance of the same FP32 transformed query and
  FP32 centroid;
* every later stage is exactly what Alg 4, the counting of Alg 6 and Alg 5
  give on the distances the GPU used: the oracle's own functions are fed the
  GPU's distances and must reproduce the centroid order, probed cells,
  retrieved counts, collision counts, histogram, threshold and candidates;
* re-rank distances are the FP32 distances of those candidates and the
  result is their top-k;
* recall@10 against FP64 ground truth stays within 0.5 points of the FP32
  form's on the 40k-point version of the 1M x 128 workload.
"""
import numpy as np
import pytest

import synthdata
from oracle import oracle as O

from gpu_parity import gpu_search, scaled_workloads, workload_index

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
# unit roundoff of the operand format, and the absolute rounding error of a
# subnormal in units of the scale (e4m3 subnormal spacing 2^-9)
U_FMT = {"bf16": 2.0 ** -8, "fp8": 2.0 ** -4}
SUB_FMT = {"bf16": 0.0, "fp8": 2.0 ** -10}
FP8_RANGE = np.float32(240.0)


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def cdist_bound(x, C, form, sx, sc, kterms):
    """Bound on |D_gpu - D| for the query half x (h,) and centroids C (l, h),
    all FP64 copies of the FP32 values; sx, sc the FP8 scales (1 for BF16);
    kterms the number of terms the matrix core accumulates."""
    u, sub = U_FMT[form], SUB_FMT[form]
    ax, ac = np.abs(x), np.abs(C)
    ex = u * ax + sub * sx + U32 * ax      # operand rounding (+ the division by the scale)
    ec = u * ac + sub * sc + U32 * ac
    conv = (ac * ex + ax * ec + ex * ec).sum(1)
    prod = ((ax + ex) * (ac + ec)).sum(1)
    nx, nc = float((x * x).sum()), (C * C).sum(1)
    cross = conv + gamma(kterms) * prod + 2 * U32 * prod
    return 2.0 * cross + gamma(x.size) * (nx + nc) + 2 * U32 * (nx + nc + 2 * prod)


def _cases():
    W = synthdata.WORKLOADS
    return [W["tiny-gmm-20k-d128"].scaled("tiny-gmm-20k-d128-q24", n=20_000, nq=24)] + scaled_workloads()


@pytest.fixture(scope="module")
def taco_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24919_amd as taco
    taco.load_library()
    return taco


FIELDS = ("qt", "cdist", "corder", "cells", "ncells", "retrieved", "sc", "hist", "last", "ncand", "cand",
          "cand_dist")


@pytest.mark.parametrize("form", ["bf16", "fp8"])
@pytest.mark.parametrize("w", _cases(), ids=lambda w: w.name)
def test_cdist_mfma_bound_and_downstream_exact(taco_mod, w, form):
    t = taco_mod
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    oidx = O.OracleIndex(path)
    alpha, beta, k = w.alphas[-1], w.beta, w.k
    print(f"[cdist {form}] {w.name} alpha={alpha}", flush=True)
    idx = t.Index(path, 0)
    try:
        idx.set_option(t.TC_OPT_CDIST_PRECISION, t.TC_CDIST_BF16 if form == "bf16" else t.TC_CDIST_FP8)
        g = gpu_search(idx, Q, k, alpha, beta, FIELDS)
    finally:
        idx.close()
    Ns, s, h1, l, n, M = oidx.Ns, oidx.s, oidx.h1, oidx.l, oidx.n, oidx.M
    C1, C2 = oidx.centroids(0).astype(np.float64), oidx.centroids(1).astype(np.float64)
    offs, ids = oidx.offsets(), oidx.ids()
    A, R = O.budget_A(alpha, n), O.budget_R(beta, n)
    kterms = (M + 31) // 32 * 32
    worst = 0.0
    for qi in range(Q.shape[0]):
        r = oidx.query(Q[qi], alpha, beta, k)
        assert np.array_equal(g["qt"][qi].view(np.uint32), r["qt"].view(np.uint32)), "q' bits"
        x = g["qt"][qi].astype(np.float64)
        sc_counts = np.zeros(n, np.int64)
        for j in range(Ns):
            xj = g["qt"][qi][j * s:(j + 1) * s]
            sx = float(np.float32(np.abs(xj).max()) / FP8_RANGE) if np.abs(xj).max() > 0 else 1.0
            cmax = max(np.abs(C1[j]).max(), np.abs(C2[j]).max())
            scj = float(np.float32(cmax) / FP8_RANGE) if cmax > 0 else 1.0
            if form == "bf16":
                sx = scj = 1.0
            halves = [(x[j * s:j * s + h1], C1[j]), (x[j * s + h1:(j + 1) * s], C2[j])]
            for h, (xh, Ch) in enumerate(halves):
                exact = ((xh[None, :] - Ch) ** 2).sum(1)
                gd = g["cdist"][qi, j, h].astype(np.float64)
                bnd = cdist_bound(xh, Ch, form, sx, scj, kterms)
                err = np.abs(gd - exact)
                assert np.all(err <= bnd), (f"{w.name} q{qi} j{j} h{h}: error {err.max()} > bound "
                                            f"{bnd[np.argmax(err - bnd)]}")
                worst = max(worst, float((err / np.maximum(bnd, 1e-30)).max()))
            # Alg 4 on the GPU's own distances
            D1, D2 = g["cdist"][qi, j, 0], g["cdist"][qi, j, 1]
            i1, i2 = O.argsort(D1), O.argsort(D2)
            assert np.array_equal(g["corder"][qi, j, 0], i1) and np.array_equal(g["corder"][qi, j, 1], i2)
            sizes = (offs[j, 1:] - offs[j, :-1]).astype(np.int64)
            cells, got = O.probe(D1, i1, D2, i2, sizes, A)
            assert g["ncells"][qi, j] == len(cells)
            assert np.array_equal(g["cells"][qi, j, :len(cells)], cells)
            assert g["retrieved"][qi, j] == got
            for c in cells:
                sc_counts[ids[j, offs[j, c]:offs[j, c + 1]]] += 1
        # counting, Alg 5 and the candidates on those cells
        assert np.array_equal(g["sc"][qi].astype(np.int64), sc_counts)
        hist, last, cand = O.select(sc_counts.astype(np.uint8), Ns, R)
        assert np.array_equal(g["hist"][qi], hist) and int(g["last"][qi]) == last
        nc = int(g["ncand"][qi])
        assert nc == len(cand)
        gc = g["cand"][qi, :nc]
        order = np.argsort(gc, kind="stable")
        assert np.array_equal(gc[order], cand)
        # re-rank: FP32 distances of the candidates, then their top k
        d64 = ((X[cand].astype(np.float64) - Q[qi].astype(np.float64)) ** 2).sum(1)
        tol = (oidx.d + 4) * U32 * d64 + 1e-30
        gdist = g["cand_dist"][qi, :nc][order].astype(np.float64)
        assert np.all(np.abs(gdist - d64) <= tol)
        top = np.lexsort((cand, d64))[:k]
        kth = d64[top[-1]]
        gi = g["ids"][qi][: len(top)]
        assert np.allclose(g["dists"][qi][: len(top)], d64[top], rtol=(oidx.d + 4) * U32 * 2)
        diff = set(gi.tolist()) ^ set(cand[top].tolist())
        pos = {int(c): i for i, c in enumerate(cand)}
        for i in diff:
            assert abs(d64[pos[int(i)]] - kth) <= 4 * (oidx.d + 4) * U32 * kth, "id differs beyond a tie"
    print(f"[cdist {form}] {w.name}: largest error / bound = {worst:.3f}", flush=True)
    oidx.close()


@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_cdist_mfma_recall_loss(taco_mod, form):
    t = taco_mod
    w = synthdata.WORKLOADS["gmm-int-1m-d128"].scaled("gmm-int-40k-d128-q400", n=40_000, nq=400)
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    gt = O.bruteforce(X, Q, w.k)
    rec = {}
    for name, val in (("fp32", t.TC_CDIST_FP32), (form, t.TC_CDIST_BF16 if form == "bf16" else t.TC_CDIST_FP8)):
        idx = t.Index(path, 0)
        idx.set_option(t.TC_OPT_CDIST_PRECISION, val)
        out = {}
        for a in w.alphas:
            g = gpu_search(idx, Q, w.k, a, w.beta)
            out[a] = O.recall_at_k(g["ids"], gt[1], X, Q, w.k)
        idx.close()
        rec[name] = out
    print(f"[cdist {form}] recall@10 fp32 {rec['fp32']} {form} {rec[form]}", flush=True)
    for a in w.alphas:
        assert rec[form][a] >= rec["fp32"][a] - 0.005, (a, rec)


def test_profiling_with_cdist_form(taco_mod):
    """Every kernel's timing reads back with the MFMA form on (its launches
    sit between the transform's and the probe's)."""
    t = taco_mod
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"]
    X, Q = synthdata.base_and_queries(w)
    idx = t.Index(workload_index(w, X), 0)
    try:
        idx.set_option(t.TC_OPT_CDIST_PRECISION, t.TC_CDIST_FP8)
        idx.set_option(t.TC_OPT_PRECISION, t.TC_BF16)
        idx.set_option(t.TC_OPT_PROFILE, 1)
        idx.profile_reset()
        gpu_search(idx, Q, w.k, 0.05, w.beta)
        got = {k: idx.kernel_time(k) for k in t.KERNELS}
    finally:
        idx.close()
    for k in ("transform", "cdist", "probe", "count", "select", "rerank", "recheck"):
        assert got[k][1] >= 1 and got[k][0] > 0.0, (k, got[k])
    assert got["topk"][1] >= 1  # the bounds; the final top-k runs inside the re-check
