"""Host-side pieces of bench.py: the recall-frontier read-out, the kernel
name mapping and the counter scaling (no GPU)."""
import csv
import json

import pytest

import bench


def test_qps_at_recall_frontier():
    pts = [dict(recall=0.90, qps=1000.0), dict(recall=0.97, qps=400.0), dict(recall=0.99, qps=300.0)]
    # interpolation between the fast point below and the slow point above
    v = bench.qps_at_recall(pts, 0.95)
    assert v == pytest.approx(400.0 + (0.97 - 0.95) / (0.97 - 0.90) * 600.0)
    # a point at or above the target that is faster wins
    pts.append(dict(recall=0.96, qps=900.0))
    assert bench.qps_at_recall(pts, 0.95) >= 900.0
    assert bench.qps_at_recall([dict(recall=0.5, qps=1.0)], 0.95) is None


def test_recall_of_per_query_k_on_a_sample_shorter_than_the_ground_truth():
    """The oracle's single-thread sample covers fewer queries than the
    ground truth: recall is read on the sample's rows only."""
    import numpy as np
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 3)).astype(np.float32)
    Q = rng.standard_normal((9, 3)).astype(np.float32)
    d = ((Q[:, None, :].astype(np.float64) - X[None].astype(np.float64)) ** 2).sum(2)
    order = np.argsort(d, axis=1)
    gt = {10: np.sort(d, 1)[:, 9], 1: np.sort(d, 1)[:, 0]}
    k_q = np.array([10, 1, 10, 1, 10], np.int32)  # a 5-query sample of the 9
    ids = np.full((5, 10), -1, np.int64)
    for i in range(5):
        ids[i, :k_q[i]] = order[i, :k_q[i]]
    assert bench.recall_of(ids, gt, X, Q[:5], 10, k_q) == pytest.approx(1.0)
    ids[0, 0] = order[0, 20]  # one miss among the three recall@10 queries
    assert bench.recall_of(ids, gt, X, Q[:5], 10, k_q) == pytest.approx((1.0 - 1.0 / 30) * 3 / 5 + 2 / 5)


def test_short_kernel_names():
    f = bench.short_kernel_name
    assert f("void taco::k_count_select<4>(taco::FuseArgs)") == "count_select"
    assert f("void taco::k_count<8>(taco::CountArgs, unsigned int*)") == "count"
    assert f("void taco::k_count<4, false, 1, false>(taco::CountArgs, unsigned int*)") == "count"
    assert f("void taco::k_count<4, false, 2, true>(taco::CountArgs, unsigned int*)") == "recount"
    assert f("taco::k_list_select(taco::ListArgs, unsigned int*, int, long)") == "list_select"
    assert f("taco::k_qbytes(float const*, int, int, unsigned int*)") == "qbytes"
    assert f("taco::k_query_order(int const*, int, int, int, int*)") == "query_order"
    assert f("taco::k_flatten_cells(int const*, int const*, int, int, int*, unsigned int*)") == "flatten"
    assert f("taco::k_select(taco::SelectArgs, int)") == "select"
    assert f("void taco::k_rerank16<16, true>(float const*)") == "rerank"
    assert f("void taco::k_rerank<16, true>(float const*)") == "rerank"
    assert f("void taco::k_recheck_topk<16, true>(float const*)") == "recheck"
    assert f("void taco::k_stream_topk<16, true, 4>(float const*, int)") == "stream"
    assert f("taco::k_topk_queued(int const*, float const*)") == "stream"
    assert f("taco::k_topk(int const*, float const*)") == "topk"
    assert f("void taco::k_rerank8<8, true, true>(float const*)") == "rerank"
    assert f("void taco::k_cdist_mfma<true>(float const*)") == "cdist"
    assert f("void taco::bld::(anonymous namespace)::k_km_assign<8>(taco::bld::KmArgs, int)") == "build_km_assign"
    assert f("taco::bld::(anonymous namespace)::k_jacobi(double const*, int, int)") == "build_jacobi"
    assert f("void taco::k_count_codes<4, 8>(unsigned short const*, long)") == "count_codes"
    assert f("taco::k_sub_select(float const*, long, int, long, unsigned long*)") == "sub_select"
    assert f("__amd_rocclr_copyBuffer") is None


def _write_pmc(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(rows):
            w.writerow([i, name, counter, v])


def test_summarize_traffic_scales_by_copy(tmp_path):
    kib = 1 << 20  # a 1 GiB copy read as exactly 1 GiB
    _write_pmc(tmp_path / "f.csv", "FETCH_SIZE",
               [("__amd_rocclr_copyBuffer", kib / 2), ("__amd_rocclr_copyBuffer", 4.0),
                ("void taco::k_count<4>(taco::CountArgs, unsigned int*)", 100.0),
                ("void taco::k_count<4>(taco::CountArgs, unsigned int*)", 300.0)])
    _write_pmc(tmp_path / "w.csv", "WRITE_SIZE",
               [("__amd_rocclr_copyBuffer", kib),
                ("void taco::k_count<4>(taco::CountArgs, unsigned int*)", 50.0)])
    line = dict(config=dict(workload="w", alpha=0.05, path="tuned", tuned_config="x"))
    (tmp_path / "b.json").write_text("log\n" + json.dumps(line) + "\n")
    out = tmp_path / "t.json"
    bench.summarize_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.json"),
                            str(out), "cmd")
    rec = json.loads(out.read_text())["records"][0]
    # the copy's fetch read half its size: fetch counts are doubled
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    c = rec["kernels"]["count"]
    assert c["dispatches"] == 2
    assert c["hbm_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2 + 50.0 * 1024)


def test_traffic_is_matched_to_the_launch_configuration(tmp_path, monkeypatch):
    """A traffic record serves only runs with its own launch configuration
    and sources; summaries of two configurations sit side by side."""
    kib = 1 << 20
    _write_pmc(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", kib / 2),
                                                 ("void taco::k_count<4>(taco::CountArgs)", 10.0),
                                                 ("void taco::k_probe<4>(float const*)", 3.0)])
    _write_pmc(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", kib),
                                                 ("void taco::k_count<4>(taco::CountArgs)", 1.0),
                                                 ("void taco::k_probe<4>(float const*)", 1.0)])
    (tmp_path / "profiles").mkdir()
    out = tmp_path / "profiles" / "traffic_w.json"
    for W in (131072, 262144):
        line = dict(config=dict(workload="w", path="fp8",
                                tuned_config=f"best W={W} mode=3 qpw=8 rr=8 precision=1 cqpw=32 nt=768 ms=7.7"))
        (tmp_path / "b.json").write_text(json.dumps(line) + "\n")
        bench.summarize_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.json"),
                                str(out), "cmd")
    assert len(json.loads(out.read_text())["records"]) == 2
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: json.loads(out.read_text())["records"][0]["source_hash"])
    run = "cached key W=262144 mode=3 qpw=8 rr=8 precision=1 cqpw=32 nt=768 (tuned at alpha=0.002)"
    assert bench.traffic_from_profiles("w", "count", run) == pytest.approx(10.0 * 1024 * 2 + 1024)
    assert bench.traffic_from_profiles("w", "count", run.replace("nt=768", "nt=1024")) is None
    assert bench.traffic_from_profiles("w", "count", None) is None
    # the count's traffic does not depend on the probe or re-rank settings;
    # other kernels need the whole configuration to agree
    other = run.replace("qpw=8", "qpw=16").replace("rr=8", "rr=32")
    assert bench.traffic_from_profiles("w", "count", other) == pytest.approx(10.0 * 1024 * 2 + 1024)
    assert bench.traffic_from_profiles("w", "probe", other) is None
    assert bench.traffic_from_profiles("w", "probe", run) == pytest.approx(3.0 * 1024 * 2 + 1024)
    # a record serves only its own bench path (precision forms, selection rule)
    assert bench.traffic_from_profiles("w", "count", run, "fp8") == pytest.approx(10.0 * 1024 * 2 + 1024)
    assert bench.traffic_from_profiles("w", "count", run, "fp8_fixed") is None
    monkeypatch.setattr(bench, "source_hash", lambda: "other")
    assert bench.traffic_from_profiles("w", "count", run) is None


def test_paths_set_their_selection_rule_and_forms():
    """Each bench path sets its selection rule (fp8_fixed: the fixed budget
    on the fp8 path's options) before tuning."""
    import types
    import paper_2603_24919_amd as taco

    class FakeIndex:
        def __init__(self):
            self.opts = {}

        def set_option(self, opt, val):
            self.opts[opt] = val

    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(mem_get_info=lambda dev: (10 << 30, 20 << 30)))
    got = {}
    for pname in ("fp32", "fp8", "fp8_fixed"):
        idx = FakeIndex()
        bench.configure_path(taco, fake_torch, idx, pname, None, 100)
        got[pname] = idx.opts
    assert got["fp32"][taco.TC_OPT_SELECT_RULE] == taco.TC_RULE_PRINTED
    assert got["fp8"][taco.TC_OPT_SELECT_RULE] == taco.TC_RULE_PRINTED
    assert got["fp8_fixed"][taco.TC_OPT_SELECT_RULE] == taco.TC_RULE_FIXED
    same = {k: v for k, v in got["fp8"].items() if k != taco.TC_OPT_SELECT_RULE}
    assert same == {k: v for k, v in got["fp8_fixed"].items() if k != taco.TC_OPT_SELECT_RULE}
    assert got["fp8"][taco.TC_OPT_CDIST_PRECISION] == taco.TC_CDIST_FP8
    assert got["fp8"][taco.TC_OPT_MAX_BATCH] == 100 and taco.TC_OPT_MAX_BATCH not in got["fp32"]
