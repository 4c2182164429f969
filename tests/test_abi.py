"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/taco.h
declares, and reject bad arguments and bad index files on the host before
touching any device.
"""
import os
import re

import numpy as np
import pytest

import paper_2603_24919_amd as taco

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "taco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    L = taco.load_library()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_binding_names_match_the_c_abi():
    for name in _declared():
        assert callable(getattr(taco, name)), name


def test_missing_file_is_tc_eio():
    with pytest.raises(taco.TacoError) as e:
        taco.tc_load_index("/nonexistent/dir/index.tcx", 0)
    assert e.value.code == taco.TC_EIO
    assert "cannot open" in taco.tc_last_error()


def _rebuild_checksum(blob: bytes) -> bytes:
    h = 14695981039346656037
    for b in blob[:-8]:
        h ^= b
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return blob[:-8] + h.to_bytes(8, "little")


def test_bad_index_files_are_tc_eformat(tiny_index, tmp_path):
    raw = open(tiny_index["path"], "rb").read()
    cases = {
        "flip": raw[:4000] + bytes([raw[4000] ^ 0x10]) + raw[4001:],
        "trunc": raw[:len(raw) // 2],
        "magic": b"TACOIDX9" + raw[8:],
        "header_only": raw[:100],
    }
    # Valid checksum but contents the kernels cannot accept: an id out of
    # range inside the first cell list.
    w = tiny_index["w"]
    K = w.l * w.l
    off_ids = 128 + 4 * (w.d + w.d * w.M + 2 * w.Ns * w.l * (w.s // 2)) + 8 * w.Ns * (K + 1)
    bad = bytearray(raw)
    bad[off_ids:off_ids + 4] = (w.n + 5).to_bytes(4, "little")
    cases["id_range"] = _rebuild_checksum(bytes(bad))
    # Ns above the kernels' limit of 16
    big = bytearray(raw)
    big[28:32] = (17).to_bytes(4, "little")
    cases["ns17"] = _rebuild_checksum(bytes(big))
    for name, blob in cases.items():
        p = tmp_path / f"{name}.tcx"
        p.write_bytes(blob)
        with pytest.raises(taco.TacoError) as e:
            taco.tc_load_index(str(p), 0)
        assert e.value.code == taco.TC_EFORMAT, (name, taco.tc_last_error())


def test_null_index_and_bad_options_rejected():
    L = taco.load_library()
    assert L.tc_search(None, None, 1, 10, 0.1, 0.1, None, None, None) == taco.TC_EINVAL
    assert L.tc_set_option(None, taco.TC_OPT_PROFILE, 1) == taco.TC_EINVAL
    assert L.tc_index_info(None, None, None, None, None, None) == taco.TC_EINVAL
    assert L.tc_kernel_time(None, b"count", None, None) == taco.TC_EINVAL
    L.tc_free_index(None)  # no-op
    assert "NULL" in taco.tc_last_error()


def _header_enums():
    src = open(os.path.join(ROOT, "include", "taco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {}
    for body in re.findall(r"enum\s+\w+\s*\{(.*?)\}", src, flags=re.S):
        for name, v in re.findall(r"\b(TC_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            vals[name] = int(v)
    return vals


def test_binding_constants_match_the_header():
    vals = _header_enums()
    assert len(vals) >= 25
    for name, v in vals.items():
        assert getattr(taco, name) == v, name


def test_kernel_names_match_the_header():
    src = open(os.path.join(ROOT, "include", "taco.h")).read()
    doc = src[src.index("Kernel timing"):src.index("int tc_kernel_time")]
    assert tuple(re.findall(r'"([a-z_]+)"', doc)) == taco.KERNELS
