"""Host-side part of the GPU index build, through the C-ABI (no GPU needed).

Alg 2 (eigensystem allocation, Section 3.2) runs in the library's host code:
its column order must equal the oracle's, and the printed hand cases.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def taco_mod():
    import paper_2603_24919_amd as taco
    taco.load_library()
    return taco


def _flat(buckets):
    return [e for b in buckets for e in b]


def test_alg2_golden_cases(taco_mod):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "alg2_allocation.json")))
    for case in g["cases"]:
        cols = taco_mod.tc_build_allocate(np.array(case["evals"], float), case["Ns"], case["s"])
        assert list(cols) == _flat(case["buckets"]), case


@pytest.mark.parametrize("seed", range(40))
def test_alg2_matches_oracle_on_random_spectra(taco_mod, seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(2, 200))
    Ns = int(rng.integers(1, 17))
    s = int(rng.integers(1, max(2, d // Ns) + 1))
    if Ns * s > d:
        s = d // Ns
    if s < 1:
        Ns, s = 1, d
    kind = seed % 4
    if kind == 0:
        ev = rng.exponential(1.0, d)
    elif kind == 1:
        ev = np.arange(d, 0, -1, dtype=float) ** -1.2          # power-law spectrum
    elif kind == 2:
        ev = np.repeat(rng.exponential(1.0, (d + 3) // 4), 4)[:d]  # exact ties
    else:
        ev = rng.exponential(1.0, d) * 10.0 ** rng.integers(-20, 3, d)  # hits the floor
    ev = np.sort(ev)[::-1].copy()
    want = _flat(O.eigensystem_allocation(ev, Ns, s))
    got = taco_mod.tc_build_allocate(ev, Ns, s)
    assert list(got) == want


def test_alg2_rejects_bad_shapes(taco_mod):
    with pytest.raises(taco_mod.TacoError):
        taco_mod.tc_build_allocate(np.ones(4), 3, 2)  # Ns*s > d
    with pytest.raises(taco_mod.TacoError):
        taco_mod.tc_build_allocate(np.zeros(4), 2, 2)  # no positive eigenvalue


def _rc(taco_mod, fn, *args):
    rc = getattr(taco_mod.load_library(), fn)(*args)
    return rc, taco_mod.tc_last_error()


def test_build_entry_points_reject_bad_arguments_before_any_device_work(taco_mod):
    import ctypes as C
    init = np.zeros(2 * 8 * 50, np.int64)
    fake = C.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    out = C.c_void_p()
    # NULL base
    rc, msg = _rc(taco_mod, "tc_build_index", None, 1000, 128, 8, 16, 50, 20, init.ctypes.data, None, 0,
                  0, None, None, 0, C.byref(out), None)
    assert rc == taco_mod.TC_EINVAL and "NULL" in msg
    # Ns * s > d
    rc, msg = _rc(taco_mod, "tc_build_index", fake, 1000, 64, 8, 16, 50, 20, init.ctypes.data, None, 0,
                  0, None, None, 0, C.byref(out), None)
    assert rc == taco_mod.TC_EINVAL
    # a seed position outside the sample
    bad = init.copy()
    bad[5] = 1000
    rc, msg = _rc(taco_mod, "tc_build_index", fake, 1000, 128, 8, 16, 50, 20, bad.ctypes.data, None, 0,
                  0, None, None, 0, C.byref(out), None)
    assert rc == taco_mod.TC_EINVAL and "seed" in msg
    # mean without B
    m = np.zeros(128, np.float32)
    rc, msg = _rc(taco_mod, "tc_build_index", fake, 1000, 128, 8, 16, 50, 20, init.ctypes.data, None, 0,
                  0, m.ctypes.data, None, 0, C.byref(out), None)
    assert rc == taco_mod.TC_EINVAL
    # training rows out of range
    train = np.array([0, 5, 2000] + list(range(10, 60)), np.int64)
    rc, msg = _rc(taco_mod, "tc_build_kmeans", fake, 1000, 128, 8, 16, 50, 1, init.ctypes.data,
                  train.ctypes.data, train.size, fake, fake, None)
    assert rc == taco_mod.TC_EINVAL and "training row" in msg
    # halves wider than 32 (s = 66)
    rc, msg = _rc(taco_mod, "tc_build_kmeans", fake, 1000, 132, 2, 66, 4, 1, init.ctypes.data, None, 0,
                  fake, fake, None)
    assert rc == taco_mod.TC_EINVAL
    # IMI with more than 4096 cells, and the eigensolver beyond 4096
    assert _rc(taco_mod, "tc_build_imi", fake, 1000, 2, 65, fake, fake, None)[0] == taco_mod.TC_EINVAL
    assert _rc(taco_mod, "tc_build_eigen", fake, 4097, fake, fake, None)[0] == taco_mod.TC_EINVAL
    assert out.value is None
