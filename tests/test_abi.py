"""The C-ABI library loads and exports every symbol include/sdg.h declares
(no compute calls: this file runs without a GPU)."""
import os
import re

import pytest

import paper_1802_04516_amd as sdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdg_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_functions()
    assert decl, "no declarations found"
    assert sorted(sdg.EXPORTED) == decl


def test_library_exports_every_declared_symbol():
    L = sdg.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []


def test_struct_layouts_match_header():
    import ctypes
    # sdg_sizes: 8 int32, 7 int64, 1 double, 8 doubles, 2 int64, 4 int32, 21 doubles, 2 int64
    assert ctypes.sizeof(sdg.Sizes) == 8 * 4 + 7 * 8 + 8 + 8 * 8 + 2 * 8 + 4 * 4 + 21 * 8 + 2 * 8 + 2 * 4 + 3 * 8 + 2 * 4
    assert ctypes.sizeof(sdg.SolveOpts) == 4 + 4 + 8 + 4 * 4 + 8 + 4 + 4
    assert ctypes.sizeof(sdg.SolveInfo) == 4 * 4 + 2 * 8


def test_create_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_create(0)
    assert ei.value.code == sdg.SDG_EDEVICE


def test_null_context_is_rejected():
    L = sdg.lib()
    assert L.sdg_set_discretization(None, 1, 0, 0, 0.1) == sdg.SDG_EINVAL
    assert b"null" in L.sdg_last_error()
    L.sdg_destroy(None)  # NULL-safe
