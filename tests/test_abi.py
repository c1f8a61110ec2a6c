"""The C ABI library loads and exports every symbol include/dgnn.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_names():
    hdr = open(os.path.join(ROOT, "include", "dgnn.h")).read()
    return set(re.findall(r"^(?:int|void|size_t)\s+(\w+)\(", hdr, re.M))


def test_library_exports_every_declared_symbol():
    from paper_2207_11571_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libdgnn.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _header_names()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2207_11571_amd import binding
    assert set(binding.SIGNATURES) == _header_names()


def test_struct_layouts_match_header_sizes():
    from paper_2207_11571_amd import binding
    assert ctypes.sizeof(binding.dg_params) == 16 + 8 * 8
    assert ctypes.sizeof(binding.solve_request) == 4 * 8 + 4 * 4 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(binding.solve_status) == 8 + 16 + 8 + 8 * 4 + 8 + 8


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2207_11571_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        binding.lib()
