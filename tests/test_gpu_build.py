"""GPU index build (Alg 1-3, Sections 3.2 and 4.1) vs the CPU oracle, through
the C-ABI.

Bit-exact: the transform of the base, the k-means centroids and labels of
every half-subspace (from the same transformed base, seeds and sample), the
IMI lists, and -- given the oracle's mean and B -- the whole index file.
Within tolerance (different but fixed FP64 summation orders): mean and
covariance to 1e-10 of the largest magnitude; eigenvalues to 1e-10 of the
largest; eigenvectors to 1e-7 where the spectral gap makes them well defined,
plus the invariants cov V = V diag(evals) and V^T V = I.
"""
import hashlib
import os

import numpy as np
import pytest

import synthdata
from oracle import oracle as O

from gpu_parity import workload_index

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
def tiny():
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"]
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    return dict(w=w, X=X, Q=Q, path=path, oidx=O.OracleIndex(path))


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _host(t):
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# Alg 1: mean and covariance, spectral decomposition, transform
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(20000, 128), (1001, 40), (2, 3), (70001, 7), (3000, 960)])
def test_stats_match_oracle(taco_mod, tiny, n, d):
    print(f"[stats] n={n} d={d}", flush=True)
    if (n, d) == (20000, 128):
        X = tiny["X"]
    else:
        X = np.random.default_rng(n + d).normal(3.0, 2.0, (n, d)).astype(np.float32)
    mean, cov = taco_mod.tc_build_stats(_dev(X))
    m0, c0 = O.mean_cov(X)
    m, c = _host(mean), _host(cov)
    assert np.max(np.abs(m - m0)) <= 1e-10 * max(np.max(np.abs(m0)), 1e-300)
    assert np.max(np.abs(c - c0)) <= 1e-10 * np.max(np.abs(c0))
    assert np.array_equal(c, c.T)


def _check_eigen(cov, ev, V, ref=None):
    d = cov.shape[0]
    scale = np.max(np.abs(cov))
    assert np.all(np.diff(ev) <= 0), "eigenvalues not descending"
    assert np.max(np.abs(cov @ V - V * ev[None, :])) <= 1e-10 * scale
    assert np.max(np.abs(V.T @ V - np.eye(d))) <= 1e-12 * d
    piv = np.argmax(np.abs(V), axis=0)
    assert np.all(V[piv, np.arange(d)] > 0), "sign convention"
    if ref is not None:
        ev0, V0 = ref
        assert np.max(np.abs(ev - ev0)) <= 1e-10 * np.max(np.abs(ev0))
        gap = np.full(d, np.inf)
        gap[:-1] = np.minimum(gap[:-1], ev0[:-1] - ev0[1:])
        gap[1:] = np.minimum(gap[1:], ev0[:-1] - ev0[1:])
        ok = gap > 1e-6 * np.max(np.abs(ev0))
        assert ok.sum() >= d // 2
        assert np.max(np.abs(V[:, ok] - V0[:, ok])) <= 1e-7


def test_eigen_matches_oracle_on_workload_covariance(taco_mod, tiny):
    _, cov = O.mean_cov(tiny["X"])
    ev, V = taco_mod.tc_build_eigen(_dev(cov))
    _check_eigen(cov, _host(ev), _host(V), O.eigh_desc(cov))


@pytest.mark.parametrize("d", [1, 2, 7, 64, 127, 128])
def test_eigen_random_spd(taco_mod, d):
    rng = np.random.default_rng(d)
    A = rng.normal(size=(d, d))
    cov = A @ A.T / d + np.diag(np.linspace(1.0, 2.0, d))
    ev, V = taco_mod.tc_build_eigen(_dev(cov))
    _check_eigen(cov, _host(ev), _host(V), O.eigh_desc(cov))


def test_eigen_closed_forms(taco_mod):
    # diagonal: eigenvalues are the entries, eigenvectors the unit vectors
    diag = np.array([3.0, 9.0, 1.0, 4.0, 7.0, 2.0])
    ev, V = taco_mod.tc_build_eigen(_dev(np.diag(diag)))
    order = np.argsort(-diag, kind="stable")
    assert np.array_equal(_host(ev), diag[order])
    assert np.array_equal(_host(V), np.eye(6)[:, order])
    # [[2,1],[1,2]]: eigenvalues 3 and 1, vectors (1,1)/sqrt2 and (1,-1)/sqrt2
    ev, V = taco_mod.tc_build_eigen(_dev(np.array([[2.0, 1.0], [1.0, 2.0]])))
    r = 1 / np.sqrt(2.0)
    assert np.allclose(_host(ev), [3.0, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(_host(V), [[r, r], [r, -r]], rtol=0, atol=1e-15)


def test_eigen_rejects_large_d(taco_mod):
    import torch
    with pytest.raises(taco_mod.TacoError):
        taco_mod.tc_build_eigen(torch.eye(4097, dtype=torch.float64, device="cuda:0"))


@pytest.mark.parametrize("d", [129, 130, 256, 961])
def test_eigen_one_sided_random_spd(taco_mod, d):
    # beyond 128 dimensions: the one-sided form
    rng = np.random.default_rng(d)
    A = rng.normal(size=(d, d))
    cov = A @ A.T / d + np.diag(np.linspace(1.0, 2.0, d))
    ev, V = taco_mod.tc_build_eigen(_dev(cov))
    _check_eigen(cov, _host(ev), _host(V), O.eigh_desc(cov))


@pytest.mark.parametrize("name,n", [("aniso-1m-d960", 6000), ("zipf-1m-d256", 20000)])
def test_eigen_one_sided_on_workload_covariance(taco_mod, name, n):
    w = synthdata.WORKLOADS[name].scaled(f"{name}-n{n}", n=n, nq=0)
    X, _ = synthdata.base_and_queries(w, nq=0)
    _, cov = O.mean_cov(X)
    ev, V = taco_mod.tc_build_eigen(_dev(cov))
    _check_eigen(cov, _host(ev), _host(V), O.eigh_desc(cov))


def test_transform_bit_exact(taco_mod, tiny):
    oi = tiny["oidx"]
    X = tiny["X"]
    T = taco_mod.tc_build_transform(_dev(X), _dev(oi.mean()), _dev(oi.B()))
    assert np.array_equal(_host(T), O.transform(X, oi.mean(), oi.B()))


# ---------------------------------------------------------------------------
# Alg 3: k-means and IMI
# ---------------------------------------------------------------------------

def _oracle_kmeans_all(T, Ns, s, l, iters, init, train):
    h1 = s // 2
    cents, labs = [], []
    for j in range(Ns):
        for hf in range(2):
            off, h = (j * s, h1) if hf == 0 else (j * s + h1, s - h1)
            c, a = O.kmeans(T, off, h, l, iters, init[j, hf], train)
            cents.append(c)
            labs.append(a)
    return cents, labs


def _compare_kmeans(taco, T, Ns, s, l, iters, init, train, label):
    print(f"[kmeans] {label}", flush=True)
    cent, assign = taco.tc_build_kmeans(_dev(T), Ns, s, l, iters, init, train)
    cent, assign = _host(cent), _host(assign)
    cents, labs = _oracle_kmeans_all(T, Ns, s, l, iters, init, train)
    h1 = s // 2
    for g in range(2 * Ns):
        h = h1 if g % 2 == 0 else s - h1
        assert np.array_equal(cent[g, :, :h], cents[g]), f"{label}: centroids of half {g}"
        assert np.array_equal(assign[g], labs[g]), f"{label}: labels of half {g}"


def test_kmeans_bit_exact_tiny_workload(taco_mod, tiny):
    w, oi = tiny["w"], tiny["oidx"]
    T = O.transform(tiny["X"], oi.mean(), oi.B())
    train, init = synthdata.kmeans_seeding(w)
    _compare_kmeans(taco_mod, T, w.Ns, w.s, w.l, w.iters, init, train, "tiny")


def _clustered(n, M, seed, centers=40):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-50, 50, (centers, M))
    return (mu[rng.integers(0, centers, n)] + rng.normal(0, 6, (n, M))).astype(np.float32)


def test_kmeans_bit_exact_sample_over_several_blocks(taco_mod):
    # 3 partial-sum blocks (the last one ragged), a training sample, odd s
    n, Ns, s, l = 140_000, 2, 7, 50
    T = _clustered(n, Ns * s + 3, 11)
    rng = np.random.default_rng(12)
    train = np.sort(rng.choice(n, size=131_073, replace=False)).astype(np.int64)
    init = np.stack([np.stack([rng.choice(train.size, l, replace=False) for _ in range(2)])
                     for _ in range(Ns)]).astype(np.int64)
    _compare_kmeans(taco_mod, T, Ns, s, l, 6, init, train, "blocks+sample")


def test_kmeans_empty_cluster_and_zero_iterations(taco_mod):
    # Seeds 0 and 1 are the same point: every tie goes to centroid 0, so
    # centroid 1 is left empty and moves to the farthest unused point.
    n, Ns, s, l = 5000, 1, 8, 6
    T = _clustered(n, s, 21, centers=5)
    T[17] = T[3]
    init = np.array([[[3, 17, 100, 200, 300, 400], [3, 17, 101, 201, 301, 401]]], np.int64)
    _compare_kmeans(taco_mod, T, Ns, s, l, 4, init, None, "empty cluster")
    _compare_kmeans(taco_mod, T, Ns, s, l, 0, init, None, "zero iterations")


@pytest.mark.parametrize("n,Ns,l", [(10_007, 3, 16), (4096 * 3 + 5, 2, 64), (33, 1, 3), (4096, 4, 50)])
def test_imi_bit_exact(taco_mod, n, Ns, l):
    print(f"[imi] n={n} Ns={Ns} l={l}", flush=True)
    rng = np.random.default_rng(n * 31 + l)
    # skewed labels: some cells crowded, many empty
    a = (rng.zipf(1.5, (2 * Ns, n)) - 1) % l
    assign = a.astype(np.int32)
    offs, ids = taco_mod.tc_build_imi(_dev(assign), Ns, l)
    offs = _host(offs).view(np.uint32)
    ids = _host(ids).view(np.uint32)
    for j in range(Ns):
        o0, i0 = O.build_imi(assign[2 * j], assign[2 * j + 1], l)
        assert np.array_equal(offs[j].astype(np.uint64), o0)
        assert np.array_equal(ids[j], i0)


# ---------------------------------------------------------------------------
# Alg 1-3 end to end
# ---------------------------------------------------------------------------

def _digest(path):
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for blk in iter(lambda: f.read(1 << 24), b""):
            h.update(blk)
    return h.hexdigest()


def _gpu_build_file(taco, w, X, tmp_path, with_oracle_basis, oidx=None):
    train, init = synthdata.kmeans_seeding(w)
    kw = {}
    if with_oracle_basis:
        kw = dict(mean=oidx.mean(), B=oidx.B())
    idx = taco.Index.build(_dev(X), w.Ns, w.s, w.l, w.iters, init, train, w.seed, **kw)
    try:
        out = str(tmp_path / f"{w.name}-gpu.tcx")
        idx.save(out)
        ms = idx.stage_ms
    finally:
        idx.close()
    return out, ms


def test_build_index_file_identical_given_oracle_basis(taco_mod, tiny, tmp_path):
    out, ms = _gpu_build_file(taco_mod, tiny["w"], tiny["X"], tmp_path, True, tiny["oidx"])
    print(f"[build] stage ms {ms}", flush=True)
    assert _digest(out) == _digest(tiny["path"])


def test_build_index_full_gpu_path(taco_mod, tiny, tmp_path):
    w, X, Q = tiny["w"], tiny["X"], tiny["Q"]
    out, ms = _gpu_build_file(taco_mod, w, X, tmp_path, False)
    print(f"[build] full GPU stage ms {ms}", flush=True)
    assert np.all(ms >= 0)
    g = O.OracleIndex(out)
    o = tiny["oidx"]
    # basis: the oracle's within FP32 rounding of eigenvectors equal to 1e-7
    assert np.max(np.abs(g.mean() - o.mean())) <= 1e-5 * np.max(np.abs(o.mean()))
    assert np.max(np.abs(g.B() - o.B())) <= 1e-6
    # every point's cell is the pair of its nearest half-centroids (FP32 chain)
    T = O.transform(X, g.mean(), g.B())
    offs, ids = g.offsets(), g.ids()
    h1 = w.s // 2
    rows = np.arange(0, w.n, 97)
    for j in range(w.Ns):
        cell_of = np.empty(w.n, np.int64)
        for c in range(w.l * w.l):
            cell_of[ids[j, offs[j, c]:offs[j, c + 1]]] = c
        C1, C2 = g.centroids(0)[j], g.centroids(1)[j]
        for r in rows:
            a = int(np.argmin(O.half_dists(T[r, j * w.s:j * w.s + h1], C1)))
            b = int(np.argmin(O.half_dists(T[r, j * w.s + h1:(j + 1) * w.s], C2)))
            assert cell_of[r] == a * w.l + b
    # the GPU-built index answers queries as well as the oracle-built one
    gt = O.bruteforce(X, Q, w.k)[1]
    r_g = O.recall_at_k(g.query_batch(Q, 0.05, w.beta, w.k), gt, X, Q, w.k)
    r_o = O.recall_at_k(o.query_batch(Q, 0.05, w.beta, w.k), gt, X, Q, w.k)
    assert r_g >= r_o - 0.02, (r_g, r_o)


def test_build_index_1m_file_identical_given_oracle_basis(taco_mod, tmp_path):
    w = synthdata.WORKLOADS["gmm-int-1m-d128"]
    X, _ = synthdata.base_and_queries(w, nq=0)
    path = workload_index(w, X)
    print(f"[build] 1M index {path}", flush=True)
    out, ms = _gpu_build_file(taco_mod, w, X, tmp_path, True, O.OracleIndex(path))
    print(f"[build] 1M stage ms {ms}", flush=True)
    assert _digest(out) == _digest(path)


@pytest.mark.parametrize("name,n,kw", [
    # d = 960, s = 60 (halves of 30), l = 32: the caller passes mean and B
    ("aniso-1m-d960", 6000, {}),
    # d = 96, s = 12, l = 64 (K = 4096 cells), a training sample of 2/3 of the rows
    ("sphere-10m-d96", 150_000, {"n_train": 100_000}),
    # d = 256, Ns = 16, l = 40
    ("zipf-1m-d256", 20_000, {}),
])
def test_build_index_other_workloads_identical_given_oracle_basis(taco_mod, tmp_path, name, n, kw):
    w = synthdata.WORKLOADS[name].scaled(f"{name}-n{n}", n=n, nq=0, **kw)
    X, _ = synthdata.base_and_queries(w, nq=0)
    path = str(tmp_path / f"{w.name}-oracle.tcx")
    O.build_workload_index(w, path, X)
    print(f"[build] {w.name}: oracle index built", flush=True)
    out, ms = _gpu_build_file(taco_mod, w, X, tmp_path, True, O.OracleIndex(path))
    print(f"[build] {w.name} stage ms {ms}", flush=True)
    assert _digest(out) == _digest(path)


def test_build_index_full_gpu_path_d256(taco_mod, tmp_path):
    # every stage on the GPU beyond 128 dimensions (one-sided eigensolver)
    w = synthdata.WORKLOADS["zipf-1m-d256"].scaled("zipf-20k", n=20000, nq=50)
    X, Q = synthdata.base_and_queries(w)
    opath = str(tmp_path / "zipf-oracle.tcx")
    O.build_workload_index(w, opath, X)
    out, ms = _gpu_build_file(taco_mod, w, X, tmp_path, False)
    print(f"[build] zipf-20k full GPU stage ms {ms}", flush=True)
    g, o = O.OracleIndex(out), O.OracleIndex(opath)
    assert np.max(np.abs(g.mean() - o.mean())) <= 1e-5 * np.max(np.abs(o.mean()))
    gt = O.bruteforce(X, Q, w.k)[1]
    r_g = O.recall_at_k(g.query_batch(Q, 0.05, w.beta, w.k), gt, X, Q, w.k)
    r_o = O.recall_at_k(o.query_batch(Q, 0.05, w.beta, w.k), gt, X, Q, w.k)
    assert r_g >= r_o - 0.02, (r_g, r_o)
