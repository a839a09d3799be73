"""CPU checks of the boundary: the built library loads and exports every symbol
the header declares, and the binding's structures match the header."""

import ctypes
import os
import re

import pytest

from paper_2601_16734_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seemps_hip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"\b(smps_[a-z0-9_]+)\s*\(", text)


def test_header_and_binding_agree():
    assert sorted(set(declared_functions())) == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libseemps_hip.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # smps_strategy: int, double, int, int, double, int, int
    assert ctypes.sizeof(binding.Strategy) == 40
    assert binding.Strategy.tol.offset == 8 and binding.Strategy.sweep_tol.offset == 24
    assert ctypes.sizeof(binding.ApplyInfo) == 48


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        binding.load(str(tmp_path / "nope.so"))


def test_context_creation_without_device_is_an_error():
    lib = binding.load()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert lib.smps_ctx_create(0, None, ctypes.byref(h)) == binding.EINVAL
