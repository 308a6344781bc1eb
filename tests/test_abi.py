"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching a GPU. Runs without a GPU."""
import ctypes

import numpy as np
import pytest

from paper_2604_05885_amd import api


def test_library_exports_every_header_symbol():
    names = api.header_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(api.lib, name), name
    assert set(names) == set(api._SIGS)  # the binding covers the whole header
    assert api.lib.jz_abi_version() == 4


def test_default_opts():
    o = api.default_opts()
    assert (o.leaf_max, o.coarsen, o.n_target, o.ngr, o.key_bits) == (64, 8, 1000, 32, 0)
    assert o.sort_max == 8192
    assert o.auto_regrow == 1 and o.keep_keys == 0 and o.list_per_node == 96.0


def _build_raw(ptr, n, opts=None):
    h = ctypes.c_void_p()
    rc = api.lib.jz_build(ptr, n, None, ctypes.byref(opts) if opts else None, None,
                          ctypes.byref(h))
    return rc, h


def test_argument_validation_without_gpu():
    rc, h = _build_raw(None, -1)
    assert rc == api.JZ_E_INVALID and not h.value
    rc, h = _build_raw(None, 10)  # NULL points with n > 0
    assert rc == api.JZ_E_INVALID
    rc, h = _build_raw(None, 2 ** 31)  # n too large
    assert rc == api.JZ_E_INVALID
    for bad in (dict(leaf_max=0), dict(leaf_max=65), dict(coarsen=1), dict(ngr=0),
                dict(key_bits=22), dict(list_per_node=0.5)):
        rc, _ = _build_raw(ctypes.c_void_p(16), 10, api.default_opts(**bad))
        assert rc == api.JZ_E_INVALID, bad
        assert api.lib.jz_last_error()
    assert api.lib.jz_knn(None, 8, None, None, None) == api.JZ_E_INVALID
    assert api.lib.jz_fof(None, 0.1, None, None) == api.JZ_E_INVALID
    assert api.lib.jz_knn_fof(None, 8, None, None, 0.1, None, None, None, None) == api.JZ_E_INVALID
    st = api.Stats()
    assert api.lib.jz_tree_stats(None, ctypes.byref(st)) == api.JZ_E_INVALID
    off = np.array([0, 5, 3], dtype=np.int64)
    h = ctypes.c_void_p()
    rc = api.lib.jz_forest_build(None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2,
                                 None, None, None, ctypes.byref(h))
    assert rc == api.JZ_E_INVALID
    api.lib.jz_tree_free(None)  # ignored


def test_no_fallback_when_library_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(api, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        api._load()
