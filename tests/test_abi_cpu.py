"""The C-ABI library loads and exports every function include/mpbjac.h
declares (no compute call: this runs without a GPU)."""
import os
import re

import pytest

from paper_2407_15973_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mpbjac.h")).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_bound_symbols():
    declared = _declared()
    assert len(declared) >= 18
    assert sorted(binding.SYMBOLS) == declared


def test_library_loads_and_exports_all_symbols():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmpbjac.so not built (run __graft_entry__.build())")
    L = binding.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.bjac_abi_version() == 4
    assert L.bjac_strerror(-2).decode().startswith("a diagonal block")


def test_struct_sizes_match_header_layout():
    import ctypes as C
    assert C.sizeof(binding.bjac_csr) == 40
    assert C.sizeof(binding.bjac_policy) == 64
    assert C.sizeof(binding.bjac_solve_opts) == 48
    assert C.sizeof(binding.bjac_stats) == 88
    assert C.sizeof(binding.bjac_info) == 64
    assert C.sizeof(binding.bjac_batch_cfg) == 16
