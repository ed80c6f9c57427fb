"""The C ABI library loads, exports every entry point that include/stf.h
declares, and rejects bad arguments on the host (no GPU needed: validation
happens before any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2305_05810_amd as stf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(stf_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for must in ("stf_create_texture2d", "stf_create_sparse_grid3d", "stf_filter", "stf_shade_filter",
                 "stf_destroy", "stf_last_error"):
        assert must in names


@pytest.mark.parametrize("name", _declared())
def test_symbol_exported(name):
    L = C.CDLL(stf.LIB_PATH)
    assert hasattr(L, name), name


def test_version():
    assert "gfx950" in stf.stf_version()


def test_create_rejects_bad_sizes():
    with pytest.raises(stf.STFError) as e:
        stf.stf_create_texture2d(0, 4, 4, stf.STF_FMT_F32, [np.zeros(16, np.float32)])
    assert e.value.status == stf.STF_E_INVALID and "size" in str(e.value)
    with pytest.raises(stf.STFError) as e:
        stf.stf_create_texture2d(4, 4, 5, stf.STF_FMT_F32, [np.zeros(80, np.float32)])
    assert e.value.status == stf.STF_E_INVALID and "channels" in str(e.value)
    with pytest.raises(stf.STFError) as e:
        stf.stf_create_texture2d(4, 4, 1, 9, [np.zeros(16, np.float32)])
    assert e.value.status == stf.STF_E_INVALID and "format" in str(e.value)


def test_grid_rejects_bad_leaves():
    v = np.zeros(2 * 512, np.float32)
    cases = [np.array([[0, 0, 0], [0, 0, 0]]), np.array([[0, 0, 0], [4, 0, 0]]),
             np.array([[0, 0, 0], [16, 0, 0]]), np.array([[0, 0, 0], [-8, 0, 0]])]
    for o in cases:
        with pytest.raises(stf.STFError) as e:
            stf.stf_create_sparse_grid3d((16, 16, 16), stf.STF_FMT_F32, o, v)
        assert e.value.status == stf.STF_E_INVALID
    with pytest.raises(stf.STFError):
        stf.stf_create_sparse_grid3d((0, 16, 16), stf.STF_FMT_F32, np.zeros((0, 3)), np.zeros(0, np.float32))


def test_filter_rejects_null_texture():
    L = stf.lib()
    rc = L.stf_filter(None, None, 0, 0, 0, 0, None, None, 0, None)
    assert rc == stf.STF_E_INVALID and "NULL" in stf.stf_last_error()
    rc = L.stf_shade_filter(None, None, 0, 0, 0, 0, None, None, None)
    assert rc == stf.STF_E_INVALID


def test_destroy_null_is_noop():
    stf.lib().stf_destroy(None)
