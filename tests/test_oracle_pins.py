"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
examples of the paper's algorithms (tests/golden), closed forms, library
routines for textbook special cases, brute force on tiny inputs, and the
invariants the method guarantees.  The FP32 chain tests pin the oracle's own
evaluation-order convention with inputs whose exact results are known.
"""
import json
import math
import os

import numpy as np
import pytest

import synthdata
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Alg 2 (Eigensystem Allocation)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", _gold("alg2_allocation.json")["cases"])
def test_alg2_hand_cases(case):
    got = O.eigensystem_allocation(np.array(case["evals"], float), case["Ns"], case["s"])
    assert got == case["buckets"]


def test_alg2_partition_properties():
    rng = np.random.default_rng(1)
    for _ in range(50):
        Ns, s = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        d = Ns * s + int(rng.integers(0, 5))
        lam = np.sort(rng.uniform(0.01, 100.0, d))[::-1]
        b = O.eigensystem_allocation(lam, Ns, s)
        assert all(len(x) == s for x in b)
        assert sorted(e for x in b for e in x) == list(range(Ns * s))
        # each bucket's members are appended in descending eigenvalue order
        assert all(x == sorted(x) for x in b)


def test_alg2_greedy_matches_bruteforce_min_max_on_tiny():
    # On tiny inputs the greedy's largest bucket product equals the best
    # achievable over all partitions of the top Ns*s eigenvalues into Ns
    # buckets of s (eq. 4 of Section 3.2 restricted to eigenvector buckets),
    # for the product-balancing objective the greedy targets.
    import itertools
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(40):
        Ns, s = 2, 2
        lam = np.sort(rng.uniform(1.0, 10.0, 4))[::-1]
        b = O.eigensystem_allocation(lam, Ns, s)
        scaled = lam / lam.min()
        greedy = max(np.prod(scaled[x]) for x in b)
        best = min(max(np.prod(scaled[list(p)]), np.prod(scaled[[i for i in range(4) if i not in p]]))
                   for p in itertools.combinations(range(4), 2))
        assert greedy == pytest.approx(best, rel=1e-12)
        checked += 1
    assert checked == 40


# ---------------------------------------------------------------------------
# Alg 1 (transform): FP64 statistics, eigenvectors, distance preservation
# ---------------------------------------------------------------------------

def test_mean_cov_match_numpy():
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((3000, 12)) * rng.uniform(0.1, 5, 12) + 7).astype(np.float32)
    mean, cov = O.mean_cov(X, chunk=256)
    np.testing.assert_allclose(mean, X.astype(np.float64).mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cov, np.cov(X.astype(np.float64), rowvar=False), rtol=1e-10, atol=1e-12)


def test_eigh_desc_is_a_sorted_signed_eigensystem():
    rng = np.random.default_rng(4)
    G = rng.standard_normal((20, 20))
    A = G @ G.T
    w, V = O.eigh_desc(A)
    assert np.all(np.diff(w) <= 0)
    np.testing.assert_allclose(A @ V, V * w[None, :], atol=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(20), atol=1e-12)
    piv = np.argmax(np.abs(V), axis=0)
    assert np.all(V[piv, np.arange(20)] > 0)


def test_transform_orthonormal_and_distance_preserving(tiny_index):
    info, X = tiny_index["info"], tiny_index["X"]
    B = info["B32"].astype(np.float64)
    np.testing.assert_allclose(B.T @ B, np.eye(B.shape[1]), atol=2e-6)
    # Ns*s = d here, so B is square orthogonal: distances are preserved.
    T = O.transform(X[:200], info["mean32"], info["B32"])
    for i, j in [(0, 1), (5, 77), (100, 199), (3, 3)]:
        a = np.linalg.norm(X[i].astype(np.float64) - X[j])
        b = np.linalg.norm(T[i].astype(np.float64) - T[j])
        assert b == pytest.approx(a, rel=2e-5, abs=1e-3)


def test_transform_matches_fp64_projection_within_fp32_error(tiny_index):
    info, X = tiny_index["info"], tiny_index["X"]
    T = O.transform(X[:64], info["mean32"], info["B32"])
    E = X[:64].astype(np.float32) - info["mean32"][None, :]
    exact = E.astype(np.float64) @ info["B32"].astype(np.float64)
    # |fl(sum) - sum| <= gamma_d * sum |terms|
    bound = 129 * 2.0 ** -24 * (np.abs(E.astype(np.float64)) @ np.abs(info["B32"].astype(np.float64)))
    assert np.all(np.abs(T - exact) <= bound + 1e-30)


def test_lemma1_non_expansion_when_reducing_dimension():
    # Section 3.3, Lemma 1 upper bound: ||B^T (x - y)|| <= ||x - y|| for a
    # transform with orthonormal columns and Ns*s < d.
    rng = np.random.default_rng(5)
    X = (rng.standard_normal((2000, 24)) * np.linspace(5, 0.5, 24)).astype(np.float32)
    mean, cov = O.mean_cov(X)
    w, V = O.eigh_desc(cov)
    b = O.eigensystem_allocation(w, 3, 4)
    B32 = np.ascontiguousarray(V[:, [e for x in b for e in x]], np.float32)
    T = O.transform(X, mean.astype(np.float32), B32)
    for i in range(0, 2000, 97):
        for j in range(1, 2000, 131):
            a = np.linalg.norm(X[i].astype(np.float64) - X[j])
            t = np.linalg.norm(T[i].astype(np.float64) - T[j])
            assert t <= a * (1 + 1e-5) + 1e-4


def test_theorem2_order_preserved_when_projection_keeps_the_differences():
    # Section 3.3, Theorem 2: when the discarded directions carry (almost)
    # none of the difference vectors, neighbour order is kept.  Data living
    # in a 6-dim subspace of R^10, projected on its top 6 eigenvectors.
    rng = np.random.default_rng(6)
    Z = rng.standard_normal((500, 6)) * np.array([9, 7, 5, 4, 3, 2.0])
    Rq, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    X = (Z @ Rq[:, :6].T + 50).astype(np.float32)
    mean, cov = O.mean_cov(X)
    w, V = O.eigh_desc(cov)
    b = O.eigensystem_allocation(np.maximum(w, 1e-9), 2, 3)
    B32 = np.ascontiguousarray(V[:, [e for x in b for e in x]], np.float32)
    T = O.transform(X, mean.astype(np.float32), B32)
    q = 0
    d_orig = np.linalg.norm(X.astype(np.float64) - X[q], axis=1)
    d_new = np.linalg.norm(T.astype(np.float64) - T[q], axis=1)
    o1, o2 = np.argsort(d_orig, kind="stable"), np.argsort(d_new, kind="stable")
    gaps = np.diff(d_orig[o1])
    # compare orders where neighbours are separated by more than rounding
    ok = np.concatenate([[True], gaps > 1e-3])
    assert np.array_equal(o1[ok][:50], o2[ok][:50]) or np.allclose(d_orig[o2], d_new[o2], atol=1e-3)


# ---------------------------------------------------------------------------
# Canonical FP32 chains (the evaluation order both sides share)
# ---------------------------------------------------------------------------

def test_transform_chain_runs_t_ascending():
    # q'_0 = fl(fl(fl(2^24*1) + 1*1) + (-2^24)*1): 2^24 + 1 rounds back to
    # 2^24 (ties to even), so ascending order gives 0; descending would give 1.
    X = np.array([[2.0 ** 24, 1.0, -2.0 ** 24]], np.float32)
    B = np.ones((3, 1), np.float32)
    T = O.transform(X, np.zeros(3, np.float32), B)
    assert T[0, 0] == 0.0


def test_transform_chain_is_fused():
    # fma(1+2^-12, 1+2^-12, -1) = 2^-11 + 2^-24 exactly; an unfused
    # multiply rounds the product to 1+2^-11 first and gives 2^-11.
    a = 1.0 + 2.0 ** -12
    X = np.array([[1.0, a]], np.float32)
    B = np.array([[-1.0], [a]], np.float32)
    T = O.transform(X, np.zeros(2, np.float32), B)
    assert T[0, 0] == np.float32(2.0 ** -11 + 2.0 ** -24)


def test_half_dist_chain_is_fused_and_ascending():
    # u = x - c per term; D = fma(u2,u2, fma(u1,u1, fma(u0,u0,0))).
    a = 1.0 + 2.0 ** -12
    x = np.array([a, 0.0], np.float32)
    cent = np.array([[0.0, 0.0]], np.float32)
    D = O.half_dists(x, cent)
    assert D[0] == np.float32(a * a)  # first term: fma(u,u,0) = fl(u*u)
    x3 = np.array([4096.0, 1.0 / 64, 1.0 / 64], np.float32)
    # 4096^2 = 2^24; adding 2^-12 twice in fp32 is lost each time (ulp 2),
    # so the ascending chain returns exactly 2^24.
    D3 = O.half_dists(x3, np.zeros((1, 3), np.float32))
    assert D3[0] == np.float32(2.0 ** 24)


def test_half_dists_close_to_fp64():
    rng = np.random.default_rng(8)
    x = rng.uniform(-50, 50, 8).astype(np.float32)
    cent = rng.uniform(-50, 50, (16, 8)).astype(np.float32)
    D = O.half_dists(x, cent)
    exact = ((cent.astype(np.float64) - x.astype(np.float64)) ** 2).sum(axis=1)
    np.testing.assert_allclose(D, exact, rtol=8 * 2.0 ** -23)


def test_argsort_is_stable_ascending():
    D = np.array([3.0, 1.0, 2.0, 1.0, 3.0, 0.5], np.float32)
    assert O.argsort(D).tolist() == [5, 1, 3, 2, 0, 4]


# ---------------------------------------------------------------------------
# k-means and the IMI (Alg 3)
# ---------------------------------------------------------------------------

def test_kmeans_one_dim_hand_case():
    # 1-D half: points {0,1,2} and {10,11,12}; seeds 0 and 12.  First step:
    # assignments split at 6; means 1 and 11; fixed point thereafter.
    T = np.array([[0], [1], [2], [10], [11], [12]], np.float32)
    cent, a = O.kmeans(T, 0, 1, 2, 5, np.array([0, 5]))
    assert cent[:, 0].tolist() == [1.0, 11.0]
    assert a.tolist() == [0, 0, 0, 1, 1, 1]


def test_kmeans_ties_go_to_lower_centroid_and_empty_cluster_reseeded():
    # Point 5 is equidistant from centroids at 4 and 6: goes to centroid 0.
    T = np.array([[4], [6], [5]], np.float32)
    cent, a = O.kmeans(T, 0, 1, 2, 0, np.array([0, 1]))
    assert a.tolist() == [0, 1, 0]
    # Duplicate seeds at 0: every point ties and goes to centroid 0, which
    # moves to their mean 4; centroid 1 gets no points and is moved onto the
    # training point farthest from its assigned centroid (12, at distance 12).
    T2 = np.array([[0], [0], [12]], np.float32)
    cent2, a2 = O.kmeans(T2, 0, 1, 2, 1, np.array([0, 1]))
    assert cent2[:, 0].tolist() == [4.0, 12.0]
    assert a2.tolist() == [0, 0, 1]


def _kmeans_2d_rows():
    # Rows of a 10 x 5 matrix whose columns 2 and 3 are the half (off = 2,
    # h = 2, ld = 5); the other columns hold values that would pull every
    # result far away if they were read.  Training rows are 0, 2, 3, 5, 6, 8:
    # positions 0..5 are (0,0) (3,0) (6,0) (10,0) (6,6) (50,50); rows 1, 4,
    # 7, 9 are not in the sample.
    pts = [(0, 0), (100, 100), (3, 0), (6, 0), (-50, -50), (10, 0), (6, 6), (5, 5), (50, 50), (4, 0)]
    T = np.zeros((10, 5), np.float32)
    for i, (a, b) in enumerate(pts):
        T[i] = (1000 + i, -1000 - i, a, b, 7777)
    return T, np.array([0, 2, 3, 5, 6, 8], np.int64)


def test_kmeans_hand_case_with_column_offset_and_training_sample():
    # Worked by hand (Alg 3's clustering step, Section 4.1), l = 3 > h = 2.
    # Seeds: sample positions 0, 1, 5 -> (0,0), (3,0), (50,50).
    # Step 1: (0,0) -> c0; (3,0) (6,0) (10,0) (6,6) -> c1 ((6,6): 72 vs 45);
    #   (50,50) -> c2.  Means: c0 (0,0), c1 (25/4, 6/4), c2 (50,50).
    # Step 2: (3,0) moves to c0 (9 vs 10.5625 + 2.25); the rest stay.
    #   Means: c0 (1.5, 0), c1 (22/3, 2), c2 (50, 50).
    # Final labels of all ten rows by nearest FP32 centroid:
    #   after 1 step  (4,0) -> c1 (16 vs 5.0625 + 2.25), after 2 steps -> c0.
    T, train = _kmeans_2d_rows()
    init = np.array([0, 1, 5])
    cent1, a1 = O.kmeans(T, 2, 2, 3, 1, init, train)
    assert cent1.tolist() == [[0.0, 0.0], [6.25, 1.5], [50.0, 50.0]]
    assert a1.tolist() == [0, 2, 0, 1, 0, 1, 1, 1, 2, 1]
    cent2, a2 = O.kmeans(T, 2, 2, 3, 2, init, train)
    assert cent2.tolist() == [[1.5, 0.0], [float(np.float32(22.0 / 3.0)), 2.0], [50.0, 50.0]]
    assert a2.tolist() == [0, 2, 0, 1, 0, 1, 1, 1, 2, 0]
    # a fixed point: a third step changes nothing
    cent3, a3 = O.kmeans(T, 2, 2, 3, 3, init, train)
    assert cent3.tolist() == cent2.tolist() and a3.tolist() == a2.tolist()


@pytest.mark.parametrize("h,n,n_train", [(3, 200_000, 150_000), (8, 6_000, 2_500)])
def test_kmeans_centroids_are_means_of_their_training_points(h, n, n_train):
    # Well separated blobs, one seed in each: after the last Lloyd step every
    # centroid is the FP64 mean of the training rows labelled with it (the
    # labels cannot flip between the last step and the final pass), rounded
    # to FP32.  The sample spans several of the oracle's 65536-row blocks in
    # the first case; columns outside [off, off + h) hold other blobs.
    rng = np.random.default_rng(100 + h)
    l, ld, off = 7, h + 9, 5
    means = rng.uniform(0, 20, (l, h)) + 40.0 * np.arange(l)[:, None]
    lab = rng.integers(0, l, n)
    T = rng.uniform(-1e4, 1e4, (n, ld)).astype(np.float32)
    T[:, off:off + h] = (means[lab] + rng.normal(0, 0.5, (n, h))).astype(np.float32)
    train = np.sort(rng.choice(n, n_train, replace=False)).astype(np.int64)
    init = np.array([int(np.flatnonzero(lab[train] == c)[0]) for c in range(l)])
    cent, assign = O.kmeans(T, off, h, l, 3, init, train)
    assert np.array_equal(assign, lab)
    X = T[train, off:off + h].astype(np.float64)
    for c in range(l):
        want = X[lab[train] == c].mean(axis=0).astype(np.float32)
        np.testing.assert_array_max_ulp(cent[c], want, maxulp=1)


def test_recall_at_k_hand_case_with_ties_and_padding():
    # One-dimensional base 0, 1, 1, 2, 4 (rows 0..4); query 1 has squared
    # distances 1, 0, 0, 1, 9 and query 3 has 9, 4, 4, 1, 1.
    X = np.array([[0], [1], [1], [2], [4]], np.float32)
    Q = np.array([[1], [3]], np.float32)
    gi, gd = O.bruteforce(X, Q, 3)
    assert gi.tolist() == [[1, 2, 0], [3, 4, 1]] and gd[:, 2].tolist() == [1.0, 4.0]
    # k = 3: the third neighbour of query 1 is at distance 1, shared by rows
    # 0 and 3, so either counts; for query 3 rows 1 and 2 tie at 4.
    ids = np.array([[2, 1, 3], [4, 2, -1]])
    assert O.recall_at_k(ids, gd, X, Q, 3) == pytest.approx(5 / 6)   # 3 + 2 hits
    ids = np.array([[0, 4, -1], [-1, -1, -1]])
    assert O.recall_at_k(ids, gd, X, Q, 3) == pytest.approx(1 / 6)   # row 0 only
    # k = 1 reads the first column only, against each query's nearest distance
    gi1, gd1 = O.bruteforce(X, Q, 1)
    ids = np.array([[2, 4, 4], [4, 0, 0]])
    assert O.recall_at_k(ids, gd1, X, Q, 1) == pytest.approx(1.0)


def test_kmeans_final_assignment_is_nearest(tiny_index):
    info, X = tiny_index["info"], tiny_index["X"]
    T = O.transform(X[:3000], info["mean32"], info["B32"])
    C1 = info["C1"][2].astype(np.float64)
    s, h1 = 16, 8
    seg = T[:, 2 * s:2 * s + h1].astype(np.float64)
    d = ((seg[:, None, :] - C1[None, :, :]) ** 2).sum(axis=2)
    # labels of these rows in subspace 2, half 1, from the cell lists
    off, ids = info["offsets"][2], info["ids"][2]
    l = C1.shape[0]
    lab = np.empty(X.shape[0], np.int64)
    for c in range(l * l):
        lab[ids[off[c]:off[c + 1]]] = c // l
    a = lab[:3000]
    best = d.min(axis=1)
    assert np.all(d[np.arange(3000), a] <= best * (1 + 1e-5) + 1e-6)


def test_imi_cells_partition_points(tiny_index):
    info = tiny_index["info"]
    n = tiny_index["X"].shape[0]
    for j in range(info["offsets"].shape[0]):
        off, ids = info["offsets"][j].astype(np.int64), info["ids"][j].astype(np.int64)
        assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
        assert np.array_equal(np.sort(ids), np.arange(n))
        for c in range(len(off) - 1):
            seg = ids[off[c]:off[c + 1]]
            assert np.all(np.diff(seg) > 0)


def test_build_imi_matches_brute_grouping():
    rng = np.random.default_rng(9)
    a1, a2 = rng.integers(0, 3, 40), rng.integers(0, 3, 40)
    off, ids = O.build_imi(a1, a2, 3)
    for c in range(9):
        want = [i for i in range(40) if a1[i] * 3 + a2[i] == c]
        assert ids[off[c]:off[c + 1]].tolist() == want


# ---------------------------------------------------------------------------
# Alg 4 (Scalable Dynamic Activation)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", _gold("alg4_probe.json")["cases"])
def test_alg4_hand_cases(case):
    D1, D2 = np.array(case["D1"], np.float32), np.array(case["D2"], np.float32)
    i1, i2 = O.argsort(D1), O.argsort(D2)
    cells, got = O.probe(D1, i1, D2, i2, np.array(case["sizes"]), case["A"])
    assert cells.tolist() == case["cells"]
    assert got == case["retrieved"]


def _activation_walk(D1, i1, D2, i2, sizes, A):
    """Section 4.2's retrieval mechanics, simulated independently of the
    oracle: a priority queue holds one (key, row, column) entry per active
    row; taking a row's cell offers that row's next column, and taking the
    first cell of row r activates row r + 1.  Cells come out until the
    retrieved total reaches A."""
    import heapq
    l = len(D1)
    key = lambda r, c: np.float32(D1[i1[r]]) + np.float32(D2[i2[c]])  # noqa: E731
    queue = [(key(0, 0), 0, 0)]
    out, got = [], 0
    while queue:
        _, r, c = heapq.heappop(queue)
        cell = int(i1[r]) * l + int(i2[c])
        out.append(cell)
        got += int(sizes[cell])
        if got >= A:
            break
        if c + 1 < l:
            heapq.heappush(queue, (key(r, c + 1), r, c + 1))
        if c == 0 and r + 1 < l:
            heapq.heappush(queue, (key(r + 1, 0), r + 1, 0))
    return out, got


def test_alg4_oracle_equals_activation_walk_on_random_grids():
    # The oracle takes the cells in their sorted order (key, row, column); an
    # independent simulation of the activation queue must give the same list,
    # including under ties of the keys and FP32 rounding collisions.
    rng = np.random.default_rng(11)
    for trial in range(3000):
        l = int(rng.integers(1, 9))
        if trial % 3 == 0:   # heavy ties
            D1 = rng.integers(0, 3, l).astype(np.float32)
            D2 = rng.integers(0, 3, l).astype(np.float32)
        elif trial % 3 == 1:  # rounding collisions of the fp32 sums
            D1 = (1e7 + rng.integers(0, 4, l)).astype(np.float32)
            D2 = rng.uniform(0, 2, l).astype(np.float32)
        else:
            D1 = rng.uniform(0, 10, l).astype(np.float32)
            D2 = rng.uniform(0, 10, l).astype(np.float32)
        sizes = rng.integers(0, 5, l * l)
        if sizes.sum() == 0:
            sizes[rng.integers(0, l * l)] = 1
        A = int(rng.integers(1, sizes.sum() + 1))
        i1, i2 = O.argsort(D1), O.argsort(D2)
        c1, g1 = O.probe(D1, i1, D2, i2, sizes, A)
        c2, g2 = _activation_walk(D1, i1, D2, i2, sizes, A)
        assert c1.tolist() == c2 and g1 == g2, trial


def test_alg4_stops_at_first_prefix_reaching_budget():
    rng = np.random.default_rng(12)
    for _ in range(300):
        l = int(rng.integers(2, 7))
        D1, D2 = rng.uniform(0, 5, l).astype(np.float32), rng.uniform(0, 5, l).astype(np.float32)
        sizes = rng.integers(0, 6, l * l)
        sizes[0] += 1
        A = int(rng.integers(1, sizes.sum() + 1))
        cells, got = O.probe(D1, O.argsort(D1), D2, O.argsort(D2), sizes, A)
        s = sizes[cells]
        assert got == s.sum() and got >= A
        assert s[:-1].sum() < A            # no earlier prefix already reached A
        assert len(set(cells.tolist())) == len(cells)
        keys = D1[cells // l] + D2[cells % l]
        assert np.all(np.diff(keys) >= 0)  # ascending distance sums
        # every cell not taken has a key >= the last key taken
        rest = np.setdiff1d(np.arange(l * l), cells)
        if rest.size:
            assert np.all(D1[rest // l] + D2[rest % l] >= keys[-1])


# ---------------------------------------------------------------------------
# Alg 5 (Query-aware Candidates Selection)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", _gold("alg5_select.json")["cases"])
@pytest.mark.parametrize("rule", ["printed", "prose"])
def test_alg5_hand_cases(case, rule):
    sc = np.array(case["sc"], np.uint8)
    R = O.budget_R(case["beta"], sc.size)
    hist, last, cand = O.select(sc, case["Ns"], R, O.RULE_PRINTED if rule == "printed" else O.RULE_PROSE)
    assert hist.tolist() == case["hist"]
    assert last == case[rule]["last"]
    assert cand.tolist() == case[rule]["cand"]


def _level_scan(hist, Ns, R, rule):
    """Section 4.3's scan restated: levels are visited from Ns down with a
    running total that includes the visited level; the visited levels that
    keep within the budget each lower the threshold from Ns by one, and the
    first level that does not ends the visit."""
    import itertools
    totals = list(itertools.accumulate(int(hist[v]) for v in range(Ns, -1, -1)))
    counts = [int(hist[v]) for v in range(Ns, -1, -1)]
    within = (t <= R if rule == O.RULE_PROSE else c + t <= R for c, t in zip(counts, totals))
    return Ns - sum(1 for _ in itertools.takewhile(bool, within))


def test_alg5_threshold_equals_level_scan():
    # The oracle states the threshold as the highest level exceeding the
    # budget; the scan of Section 4.3 must give the same level, -1 included.
    rng = np.random.default_rng(17)
    for trial in range(2000):
        Ns = int(rng.integers(0, 17))
        hist = rng.integers(0, 6, Ns + 1)
        if trial % 4 == 0:
            hist[rng.integers(0, Ns + 1)] = 0
        R = int(rng.integers(0, 3 * int(hist.sum()) + 2))
        for rule in (O.RULE_PRINTED, O.RULE_PROSE):
            assert O.threshold(hist, Ns, R, rule) == _level_scan(hist, Ns, R, rule), (trial, rule)


def test_alg5_candidate_count_bounds():
    # Levels above the stopping level add up to at most R under either
    # reading; the stopping level itself is then included whole.
    rng = np.random.default_rng(13)
    for _ in range(500):
        Ns = int(rng.integers(1, 17))
        sc = rng.integers(0, Ns + 1, int(rng.integers(1, 300))).astype(np.uint8)
        R = int(rng.integers(0, sc.size + 1))
        for rule in (O.RULE_PRINTED, O.RULE_PROSE):
            hist, last, cand = O.select(sc, Ns, R, rule)
            assert hist.sum() == sc.size
            if last >= 0:
                above = hist[last + 1:].sum() if last + 1 <= Ns else 0
                assert above <= R
                assert cand.size == hist[max(last, 0):].sum()
            else:
                assert cand.size == sc.size


def test_budgets_in_double():
    assert O.budget_A(0.05, 20000) == 1000      # the double product rounds to 1000 exactly
    assert O.budget_A(0.07, 100) == 8           # 0.07*100 = 7.000000000000001 in double
    # an alpha passed through float32 is a different number: 0.05f*20000 > 1000
    assert O.budget_A(float(np.float32(0.05)), 20000) == 1001
    assert O.budget_A(0.05, 1_000_000) == 50_000
    assert O.budget_R(0.005, 20000) == 100
    assert O.budget_A(1.0, 7) == 7 and O.budget_A(1e-9, 7) == 1
    assert O.budget_R(0.0, 7) == 0 and O.budget_R(1.0, 7) == 7


# ---------------------------------------------------------------------------
# Whole query (Alg 6): invariants and the brute-force special case
# ---------------------------------------------------------------------------

def test_bruteforce_matches_full_sort():
    rng = np.random.default_rng(14)
    X = rng.integers(0, 4, (300, 5)).astype(np.float32)   # many exact ties
    Q = rng.integers(0, 4, (7, 5)).astype(np.float32)
    ids, dist = O.bruteforce(X, Q, 12)
    for i in range(7):
        dd = ((X.astype(np.float64) - Q[i]) ** 2).sum(axis=1)
        order = np.lexsort((np.arange(300), dd))[:12]
        assert ids[i].tolist() == order.tolist()
        np.testing.assert_array_equal(dist[i], dd[order])


def test_query_stage_invariants(tiny_index):
    idx, Q, w = tiny_index["idx"], tiny_index["Q"], tiny_index["w"]
    offs, cid = idx.offsets().astype(np.int64), idx.ids()
    for qi in range(0, 100, 9):
        for alpha, beta in ((0.05, 0.005), (0.01, 0.02), (0.2, 0.001)):
            r = idx.query(Q[qi], alpha, beta, 10)
            sc = r["sc"].astype(np.int64)
            assert sc.max() <= idx.Ns
            assert sc.sum() == r["retrieved"].sum()          # counts sum to the probed list sizes
            A = O.budget_A(alpha, idx.n)
            for j in range(idx.Ns):
                cells = r["cells"][j]
                sizes = offs[j, 1:] - offs[j, :-1]
                assert r["retrieved"][j] == sizes[cells].sum() >= A
                assert sizes[cells[:-1]].sum() < A
                # the activation walk of Section 4.2 on the dumped distances
                D1, D2 = r["cdist"][j, 0], r["cdist"][j, 1]
                c2, _ = _activation_walk(D1, r["corder"][j, 0], D2, r["corder"][j, 1], sizes, A)
                assert c2 == cells.tolist()
            # SC recomputed by brute force from the probed cell lists
            want = np.zeros(idx.n, np.int64)
            for j in range(idx.Ns):
                for c in r["cells"][j]:
                    want[cid[j, offs[j, c]:offs[j, c + 1]]] += 1
            assert np.array_equal(want, sc)
            assert r["hist"].tolist() == np.bincount(sc, minlength=idx.Ns + 1).tolist()
            assert r["cand"].tolist() == np.flatnonzero(sc >= r["last"]).tolist()
            # top-k is the k smallest candidates by (fp32 distance, id)
            order = np.lexsort((r["cand"], r["cand_d32"]))[:10]
            assert r["ids"][:order.size].tolist() == r["cand"][order].tolist()
            X = tiny_index["X"]
            exact = ((X[r["cand"]].astype(np.float64) - Q[qi]) ** 2).sum(axis=1)
            np.testing.assert_allclose(r["cand_d64"], exact, rtol=1e-12)
            np.testing.assert_allclose(r["cand_d32"], exact, rtol=1e-5)


@pytest.mark.parametrize("rule", [O.RULE_PRINTED, O.RULE_PROSE])
def test_alpha_beta_one_is_exact_knn(tiny_index, rule):
    idx, Q, X = tiny_index["idx"], tiny_index["Q"], tiny_index["X"]
    gi, gd = O.bruteforce(X, Q[:20], 10)
    ids, d32, d64 = idx.query_batch(Q[:20], 1.0, 1.0, 10, rule=rule, with_dists=True)
    assert np.array_equal(ids, gi)
    np.testing.assert_allclose(d64, gd, rtol=1e-12)
    np.testing.assert_allclose(d32, gd, rtol=1e-5)
    r = idx.query(Q[0], 1.0, 1.0, 10, rule=rule)
    assert np.all(r["sc"] == idx.Ns) and r["ncand"] == idx.n


def test_padding_when_fewer_candidates_than_k(tiny_index):
    idx, Q = tiny_index["idx"], tiny_index["Q"]
    r = idx.query(Q[3], 0.0001, 0.0, 1000)
    nc = r["ncand"]
    assert nc < 1000
    assert np.all(r["ids"][nc:] == -1) and np.all(np.isinf(r["d32"][nc:]))
    assert np.all(r["ids"][:nc] >= 0)


def test_batch_equals_single_and_thread_count_invariant(tiny_index):
    idx, Q = tiny_index["idx"], tiny_index["Q"]
    a = idx.query_batch(Q[:30], 0.05, 0.005, 10, nthreads=1)
    b = idx.query_batch(Q[:30], 0.05, 0.005, 10, nthreads=4)
    assert np.array_equal(a, b)
    for i in range(0, 30, 7):
        assert np.array_equal(a[i], idx.query(Q[i], 0.05, 0.005, 10, dump=False)["ids"])
    alphas = np.linspace(0.01, 0.1, 30)
    c = idx.query_batch(Q[:30], alphas, 0.005, 10)
    for i in (0, 13, 29):
        assert np.array_equal(c[i], idx.query(Q[i], alphas[i], 0.005, 10, dump=False)["ids"])


def test_rejects_bad_arguments(tiny_index):
    idx, Q = tiny_index["idx"], tiny_index["Q"]
    for a, b, k in ((0.0, 0.1, 10), (1.5, 0.1, 10), (0.1, -0.1, 10), (0.1, 1.1, 10), (0.1, 0.1, 0),
                    (0.1, 0.1, idx.n + 1), (math.nan, 0.1, 10)):
        with pytest.raises(ValueError):
            idx.query(Q[0], a, b, k)


# ---------------------------------------------------------------------------
# Index file
# ---------------------------------------------------------------------------

def test_index_file_round_trip_and_corruption(tiny_index, tmp_path):
    idx, info = tiny_index["idx"], tiny_index["info"]
    assert np.array_equal(idx.offsets(), info["offsets"])
    assert np.array_equal(idx.ids(), info["ids"])
    assert np.array_equal(idx.centroids(0), info["C1"]) and np.array_equal(idx.centroids(1), info["C2"])
    assert np.array_equal(idx.B(), info["B32"]) and np.array_equal(idx.mean(), info["mean32"])
    assert np.array_equal(idx.base(), tiny_index["X"])
    raw = open(tiny_index["path"], "rb").read()
    for name, blob in (("flip", raw[:5000] + bytes([raw[5000] ^ 1]) + raw[5001:]),
                       ("trunc", raw[:-9]), ("magic", b"X" + raw[1:]), ("empty", b"")):
        p = tmp_path / f"{name}.tcx"
        p.write_bytes(blob)
        with pytest.raises(RuntimeError):
            O.OracleIndex(str(p))


def test_workload_recipes_are_seeded_and_shaped():
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"].scaled("t", n=3000, nq=5)
    X1, Q1 = synthdata.base_and_queries(w)
    X2, Q2 = synthdata.base_and_queries(w)
    assert np.array_equal(X1, X2) and np.array_equal(Q1, Q2)
    assert X1.shape == (3000, 128) and Q1.shape == (5, 128) and X1.min() >= 0
    for name in ("gmm-int-1m-d128", "aniso-1m-d960", "sphere-10m-d96", "zipf-1m-d256"):
        ws = synthdata.WORKLOADS[name].scaled("s", n=2000, nq=3)
        X, Q = synthdata.base_and_queries(ws)
        assert X.shape == (2000, ws.d) and X.dtype == np.float32 and np.isfinite(X).all()
        if ws.recipe == "gmm_int":
            assert np.array_equal(X, np.rint(X)) and X.min() >= 0 and X.max() <= 255
        if ws.recipe == "sphere":
            np.testing.assert_allclose(np.linalg.norm(X, axis=1), 1.0, rtol=1e-5)


# ---------------------------------------------------------------------------
# The fixed-budget rule (SuCo's selection, which Section 4.3 contrasts with
# Alg 5): the floor(beta*n) highest SC-scores, ties broken by the lower id.
# ---------------------------------------------------------------------------

def test_fixed_budget_hand_case():
    sc = np.array([3, 3, 2, 2, 2, 1, 1, 0, 0, 0], np.uint8)
    # R = 3: both 3s, then the lowest id of level 2
    hist, last, cand = O.select(sc, 3, 3, O.RULE_FIXED)
    assert list(cand) == [0, 1, 2] and last == 3
    # R = 5: the whole of level 2 is taken
    assert list(O.select(sc, 3, 5, O.RULE_FIXED)[2]) == [0, 1, 2, 3, 4]
    assert O.select(sc, 3, 5, O.RULE_FIXED)[1] == 3
    # R = 8: one zero, the lowest id among them
    hist, last, cand = O.select(sc, 3, 8, O.RULE_FIXED)
    assert list(cand) == [0, 1, 2, 3, 4, 5, 6, 7] and last == 1
    # R = 0: nothing; R = n: everything
    assert O.select(sc, 3, 0, O.RULE_FIXED)[2].size == 0 and O.select(sc, 3, 0, O.RULE_FIXED)[1] == 4
    assert list(O.select(sc, 3, 10, O.RULE_FIXED)[2]) == list(range(10))


@pytest.mark.parametrize("seed", range(30))
def test_fixed_budget_properties(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    Ns = int(rng.integers(1, 17))
    sc = rng.integers(0, Ns + 1, n).astype(np.uint8)
    if seed % 3 == 0:
        sc[rng.random(n) < 0.8] = 0  # mostly unprobed points
    R = int(rng.integers(0, n + 1))
    hist, last, cand = O.select(sc, Ns, R, O.RULE_FIXED)
    assert np.array_equal(hist, np.bincount(sc, minlength=Ns + 1))
    assert cand.size == min(R, n)
    assert np.all(np.diff(cand) > 0)
    chosen = np.zeros(n, bool)
    chosen[cand] = True
    if cand.size and cand.size < n:
        assert sc[chosen].min() >= sc[~chosen].max()
        L = int(sc[chosen].min())
        # at the boundary level the chosen ids are the smallest ones
        at = np.flatnonzero(sc == L)
        k = int(np.count_nonzero(chosen & (sc == L)))
        assert np.array_equal(np.flatnonzero(chosen & (sc == L)), at[:k])
        assert last == L + 1


# ---------------------------------------------------------------------------
# SC-Linear (Section 2.3, Definitions 5 and 6): the index-free baseline
# ---------------------------------------------------------------------------

def _hand_index(tmp_path):
    g = _gold("sclinear.json")
    X = np.array(g["points"], np.float32)
    n, d = X.shape
    path = str(tmp_path / "hand.tcx")
    O.write_index(path, np.zeros(d, np.float32), np.eye(d, dtype=np.float32),
                  np.zeros((2, 1, 1), np.float32), np.zeros((2, 1, 1), np.float32),
                  np.array([[0, n], [0, n]], np.uint64), np.tile(np.arange(n, dtype=np.uint32), (2, 1)),
                  X, s=2, l=1)
    return g, X, O.OracleIndex(path)


def test_sclinear_hand_cases(tmp_path):
    g, X, idx = _hand_index(tmp_path)
    T = idx.transformed_base()
    assert np.array_equal(T, X)                      # the identity transform
    q = np.array(g["query"], np.float32)
    for c in g["cases"]:
        r = idx.sclinear(T, q, c["alpha"], c["beta"], c["k"])
        assert r["sc"].tolist() == c["sc"], c["why"]
        assert r["cand"].tolist() == c["cand"], c["why"]
        assert r["ids"].tolist() == c["ids"], c["why"]
        want = [np.inf if v is None else v for v in c["d32"]]
        assert r["d32"].tolist() == want, c["why"]
    idx.close()


def test_sclinear_invariants(tiny_index):
    # each subspace contributes exactly A collisions; every score is at most
    # Ns; beta = 1 re-ranks every point (exact k-NN); alpha = 1 makes every
    # score Ns, so the candidates are the R lowest ids.
    idx, Q, X = tiny_index["idx"], tiny_index["Q"], tiny_index["X"]
    T = idx.transformed_base()
    n, Ns = idx.n, idx.Ns
    for qi, alpha, beta in ((0, 0.05, 0.005), (7, 0.01, 0.02), (31, 0.2, 0.001)):
        r = idx.sclinear(T, Q[qi], alpha, beta, 10)
        assert int(r["sc"].astype(np.int64).sum()) == Ns * O.budget_A(alpha, n)
        assert r["sc"].max() <= Ns and r["cand"].size == O.budget_R(beta, n)
        # the candidates hold the highest scores: none left out scores more
        out = np.setdiff1d(np.arange(n), r["cand"])
        assert r["sc"][out].max() <= r["sc"][r["cand"]].min()
    gi, gd = O.bruteforce(X, Q[:5], 10)
    ids, d32 = idx.sclinear_batch(T, Q[:5], 0.03, 1.0, 10)
    assert np.array_equal(ids, gi)
    np.testing.assert_allclose(d32, gd, rtol=1e-5)
    r = idx.sclinear(T, Q[3], 1.0, 0.003, 10)
    assert np.all(r["sc"] == Ns) and r["cand"].tolist() == list(range(O.budget_R(0.003, n)))
    # one query alone and in a batch on several threads agree
    ids1, _ = idx.sclinear_batch(T, Q[:8], 0.05, 0.005, 10, nthreads=3)
    for i in range(8):
        assert idx.sclinear(T, Q[i], 0.05, 0.005, 10)["ids"].tolist() == ids1[i].tolist()


def test_sclinear_collisions_are_the_nearest_in_each_subspace(tmp_path):
    # One subspace (Ns = 1) covering the whole identity-transformed space:
    # the collisions are the A nearest points, so with beta such that R = A
    # the candidates are exactly the A nearest by (distance, id) (ties are
    # made frequent by integer coordinates).
    rng = np.random.default_rng(31)
    X = rng.integers(0, 5, (300, 4)).astype(np.float32)
    path = str(tmp_path / "one.tcx")
    O.write_index(path, np.zeros(4, np.float32), np.eye(4, dtype=np.float32),
                  np.zeros((1, 1, 2), np.float32), np.zeros((1, 1, 2), np.float32),
                  np.array([[0, 300]], np.uint64), np.arange(300, dtype=np.uint32)[None, :], X, s=4, l=1)
    idx = O.OracleIndex(path)
    T = idx.transformed_base()
    for trial in range(20):
        q = rng.integers(0, 5, 4).astype(np.float32) + np.float32(0.5) * (trial % 2)
        A = int(rng.integers(1, 300))
        alpha = A / 300.0
        r = idx.sclinear(T, q, alpha, alpha, 5)
        d = ((X.astype(np.float64) - q) ** 2).sum(1)
        want = np.sort(np.lexsort((np.arange(300), d))[:O.budget_A(alpha, 300)])
        assert r["sc"].sum() == want.size and np.array_equal(np.flatnonzero(r["sc"]), want)
    idx.close()
