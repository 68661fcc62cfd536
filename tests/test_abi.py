"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "trig.h")
LIB = os.path.join(ROOT, "paper_1411_3968_amd", "libtrig.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trig_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("trig_create", "trig_destroy", "trig_geom_load", "trig_slice", "trig_batch",
              "trig_stream_submit", "trig_stream_poll", "trig_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libtrig.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_the_abi_names():
    from paper_1411_3968_amd import trig as T
    for n in declared_functions():
        assert hasattr(T, n), n
    assert T.trig_version().startswith("libtrig")


def test_struct_sizes_match_header():
    from paper_1411_3968_amd import trig as T
    assert T.FIRE_DTYPE.itemsize == 24 and T.EVENT_DTYPE.itemsize == 32
    assert ctypes.sizeof(T.Result) == 112
    assert ctypes.sizeof(T.SliceDesc) == 48


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1411_3968_amd import trig as T
    with pytest.raises(T.TrigError):
        T.trig_create(0)


def test_oracle_is_not_used_by_the_product():
    pkg = os.path.join(ROOT, "paper_1411_3968_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle.c", ""), f
