"""The C-ABI library loads and exports every symbol its header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcpr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mcpr_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ["mcpr_fine_propagate", "mcpr_moments", "mcpr_match", "mcpr_parareal_iterate"]:
        assert n in names


def test_header_declares_reserve_and_allocation_counter():
    """The scratch is sized outside the hot path (mcpr_reserve) and the
    allocations a context makes are counted (mcpr_alloc_stats); a call on an
    unreserved shape is refused with its own status."""
    names = declared_functions()
    assert "mcpr_reserve" in names and "mcpr_alloc_stats" in names
    src = open(HEADER).read()
    assert "MCPR_E_NOT_RESERVED = -6" in src
    for k in ("INIT", "MOMENTS", "QOI", "FINE", "MATCH", "ADJOINT"):
        assert f"MCPR_RESERVE_{k}" in src


def test_library_exports_every_declared_symbol():
    from paper_2310_11365_amd import mcpr
    if not os.path.exists(mcpr.LIB_PATH):
        pytest.fail("libmcpr.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  one HIP runtime per process
    L = ctypes.CDLL(mcpr.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    L.mcpr_version.restype = ctypes.c_char_p
    assert L.mcpr_version().startswith(b"mcpr")


def test_struct_layouts_match_header():
    from paper_2310_11365_amd import mcpr
    assert ctypes.sizeof(mcpr.ProblemC) == 14 * 8 + 2 * 4 + 6 * 8 + 4 * 4 + 7 * 8 + 8 + 2 * 4
    assert ctypes.sizeof(mcpr.EnsembleC) == 32
    assert ctypes.sizeof(mcpr.InstanceC) == 32
    assert mcpr.STATS_DTYPE.itemsize == 48 and mcpr.MAP_DTYPE.itemsize == 32
