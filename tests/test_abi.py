"""The C ABI library loads and exports every symbol include/crk.h declares (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "crk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("crk_build_leaf_pairs", "crk_volume", "crk_corrections", "crk_accel_energy",
                 "sr_gravity", "crk_leaves_free", "crk_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import paper_2310_16122_amd as crk

    if not os.path.exists(crk.LIB_PATH):
        pytest.fail("libcrk.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(crk.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(crk.EXPORTS) == set(declared_symbols())


def test_last_error_returns_a_string():
    import paper_2310_16122_amd as crk

    lib = crk.load_library()
    assert isinstance(lib.crk_last_error(), bytes)


def test_library_imports_no_device_allocator():
    """The library allocates no device memory: it does not even link hipMalloc,
    hipFree or their relatives (the handle lives in the caller's workspace)."""
    import subprocess

    import paper_2310_16122_amd as crk

    if not os.path.exists(crk.LIB_PATH):
        pytest.fail("libcrk.so is not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--undefined-only", crk.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    imported = {line.split()[-1].split("@")[0] for line in out.splitlines() if line.strip()}
    for name in ("hipMalloc", "hipFree", "hipMallocAsync", "hipFreeAsync", "hipMallocManaged",
                 "hipExtMallocWithFlags", "hipHostMalloc", "hipMallocPitch", "hipMalloc3D"):
        assert name not in imported, name
