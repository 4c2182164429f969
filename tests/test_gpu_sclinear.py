"""SC-Linear on the GPU (tc_search_sclinear) against the oracle's SC-Linear:
SC-scores, level histogram and candidate sets bit-exact, re-rank distances
within 1e-5, result ids equal except at distance ties."""
import numpy as np
import pytest

import synthdata
from oracle import oracle as O

from gpu_parity import check_topk, scaled_workloads, workload_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def taco_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24919_amd as taco
    taco.load_library()
    return taco


def _compare(t, path, Q, k, alpha, beta, label):
    import torch
    oidx = O.OracleIndex(path)
    T = oidx.transformed_base()
    idx = t.Index(path, 0)
    try:
        q = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
        dump = idx.dump_buffers(Q.shape[0], ("sc", "hist", "ncand", "cand"))
        ids, dists = idx.search_sclinear(q, k, alpha, beta, dump)
        torch.cuda.synchronize()
        g = {f: v.cpu().numpy() for f, v in dump.items()}
        ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    finally:
        idx.close()
    n, Ns = oidx.n, oidx.Ns
    for qi in range(Q.shape[0]):
        r = oidx.sclinear(T, Q[qi], alpha, beta, k)
        lab = f"{label} q{qi}"
        assert np.array_equal(g["sc"][qi], r["sc"]), f"{lab}: SC-scores"
        assert np.array_equal(g["hist"][qi], np.bincount(r["sc"], minlength=Ns + 1)), f"{lab}: histogram"
        nc = int(g["ncand"][qi])
        assert nc == r["cand"].size, f"{lab}: candidate count"
        assert np.array_equal(np.sort(g["cand"][qi, :nc]), r["cand"]), f"{lab}: candidates"
        d64 = ((oidx.base()[r["cand"]].astype(np.float64) - Q[qi].astype(np.float64)) ** 2).sum(1)
        cand_d = np.full(n, np.inf)
        cand_d[r["cand"]] = d64
        check_topk(ids[qi], dists[qi], r["ids"], r["d32"], cand_d, lab)
    oidx.close()


@pytest.mark.parametrize("alpha,beta,k", [(0.05, 0.005, 10), (0.01, 0.02, 1), (0.3, 0.001, 25),
                                          (1.0, 0.003, 10), (0.02, 0.0, 5), (0.002, 1.0, 10)])
def test_sclinear_tiny(taco_mod, alpha, beta, k):
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"]
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    print(f"[sclinear tiny] alpha={alpha} beta={beta} k={k}", flush=True)
    _compare(taco_mod, path, Q[:24], k, alpha, beta, f"tiny a={alpha} b={beta}")


@pytest.mark.parametrize("w", scaled_workloads(), ids=lambda w: w.name)
def test_sclinear_workload_shapes(taco_mod, w):
    X, Q = synthdata.base_and_queries(w)
    path = workload_index(w, X)
    print(f"[sclinear {w.name}]", flush=True)
    _compare(taco_mod, path, Q[:8], 10, 0.02, 0.005, w.name)


def test_sclinear_hand_case(taco_mod, tmp_path):
    """The hand-worked six-point case of the oracle's pins, on the GPU."""
    import json
    import os
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sclinear.json")))
    X = np.array(g["points"], np.float32)
    n, d = X.shape
    path = str(tmp_path / "hand.tcx")
    O.write_index(path, np.zeros(d, np.float32), np.eye(d, dtype=np.float32),
                  np.zeros((2, 1, 1), np.float32), np.zeros((2, 1, 1), np.float32),
                  np.array([[0, n], [0, n]], np.uint64), np.tile(np.arange(n, dtype=np.uint32), (2, 1)),
                  X, s=2, l=1)
    idx = taco_mod.Index(path, 0)
    q = torch.tensor([g["query"]], dtype=torch.float32, device="cuda")
    for c in g["cases"]:
        dump = idx.dump_buffers(1, ("sc", "ncand", "cand"))
        ids, dists = idx.search_sclinear(q, c["k"], c["alpha"], c["beta"], dump)
        torch.cuda.synchronize()
        assert dump["sc"][0].cpu().numpy().tolist() == c["sc"], c["why"]
        nc = int(dump["ncand"][0])
        assert sorted(dump["cand"][0, :nc].cpu().numpy().tolist()) == c["cand"], c["why"]
        assert ids[0].cpu().numpy().tolist() == c["ids"], c["why"]
        want = [np.inf if v is None else v for v in c["d32"]]
        assert dists[0].cpu().numpy().tolist() == want, c["why"]
    idx.close()
