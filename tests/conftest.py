import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def tiny_index(tmp_path_factory):
    """Index of the 20k x 128 workload, built once by the oracle."""
    import synthdata
    from oracle import oracle as O
    w = synthdata.WORKLOADS["tiny-gmm-20k-d128"]
    X, Q = synthdata.base_and_queries(w)
    path = str(tmp_path_factory.mktemp("idx") / "tiny.tcx")
    info = O.build_workload_index(w, path, X)
    return dict(w=w, X=X, Q=Q, path=path, info=info, idx=O.OracleIndex(path))
