"""The C ABI library loads and exports every entry point include/hfcr.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfcr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hfcr_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("hfcr_create", "hfcr_destroy", "hfcr_resolve", "hfcr_detect", "hfcr_last_error",
                     "hfcr_default_opts", "hfcr_test_orient"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1409_2081_amd as hf
    if not os.path.exists(hf.LIB_PATH):
        from paper_1409_2081_amd import build
        build.build()
    L = ctypes.CDLL(hf.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(hf.EXPORTED) == _declared()


def test_default_opts_without_device():
    import paper_1409_2081_amd as hf
    o = hf.Opts()
    hf.lib().hfcr_default_opts(ctypes.byref(o))
    assert o.max_rounds == 256 and o.both_mode == 0 and o.predicate_tier == 0 and o.flags == 0


def test_struct_sizes_match_header_layout():
    import paper_1409_2081_amd as hf
    assert ctypes.sizeof(hf.Mesh) == 32
    assert ctypes.sizeof(hf.Opts) == 40
    assert ctypes.sizeof(hf.Result) == 56


def test_create_fails_cleanly_without_device():
    import torch
    import paper_1409_2081_amd as hf
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert hf.lib().hfcr_create(ctypes.byref(h), 0) == hf.HFCR_E_DEVICE
