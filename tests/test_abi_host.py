"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/sparqs.h declares, and its footprint model is sane."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "sparqs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_0-9]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    from paper_2503_15118_amd import _abi
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(_abi.lib, n)]
    assert not missing, missing
    assert set(names) == set(_abi.EXPORTED)


def test_strerror_and_footprint():
    from paper_2503_15118_amd import _abi
    assert _abi.strerror(0) == "ok"
    assert "capacity" in _abi.strerror(_abi.SS_E_CAPACITY)
    c1 = [("a", 7), ("b", 7), ("anc", 6)]
    small = _abi.required_bytes(c1, 1, 1 << 14)
    big = _abi.required_bytes(c1, 1, 1 << 20)
    # two 24-byte buffers per entry dominate (W = 1); look-back words and the
    # per-workgroup sort histograms add a few bytes per entry
    assert 48 * (1 << 20) < big - small < 53 * (1 << 20)
    c2 = [("a", 32), ("b", 32), ("c", 32), ("flag", 1)]
    b2 = _abi.required_bytes(c2, 1, 1 << 20) - _abi.required_bytes(c2, 1, 1 << 14)
    assert 64 * ((1 << 20) - (1 << 14)) < b2 < 70 * (1 << 20)


def test_layout_rejections():
    from paper_2503_15118_amd import _abi
    with pytest.raises(_abi.SSError):
        _abi.required_bytes([("a", 65)], 1, 1024)
    with pytest.raises(_abi.SSError):
        _abi.required_bytes([("a", 64)] * 5, 1, 1024)      # more than 4 key words
    with pytest.raises(_abi.SSError):
        _abi.required_bytes([("a", 8)], 0, 1024)           # no instances


def test_op_record_layout_matches_header():
    from paper_2503_15118_amd import _abi
    import workloads as wl
    import numpy as np
    rec = _abi.to_ss_ops(wl.ops_array([wl.make_op("RY", 2, qmask=4, theta=0.5, ctls=[(1, 3, 1)])]))
    raw = rec.tobytes()
    assert len(raw) == 64
    assert int.from_bytes(raw[0:2], "little") == 2          # kind
    assert raw[2] == 1                                      # nctl
    assert int.from_bytes(raw[4:8], "little") == 2          # reg
    assert int.from_bytes(raw[16:24], "little") == 4        # qmask
    assert np.frombuffer(raw[32:40], dtype=np.float64)[0] == 0.5
    assert int.from_bytes(raw[40:44], "little") == 1        # ctl[0].reg
    assert int.from_bytes(raw[44:46], "little") == 3        # ctl[0].qubit
    assert int.from_bytes(raw[46:48], "little") == 1        # ctl[0].value
