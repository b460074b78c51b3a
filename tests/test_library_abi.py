"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1701_06254_amd", "libr2p.so")


def _declared():
    hdr = open(os.path.join(ROOT, "include", "r2p.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(r2p_[a-z0-9_]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_1701_06254_amd.build import build
        build()
    return LIB


def test_header_entry_points_exported(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (r2p_[a-z0-9_]+)", out))
    declared = _declared()
    assert len(declared) >= 20
    missing = [d for d in declared if d not in exported]
    assert not missing, missing


def test_ctypes_binding_covers_header(lib_path):
    from paper_1701_06254_amd import r2p
    L = r2p.load(lib_path)
    for name in _declared():
        assert hasattr(L, name)
    assert set(r2p.EXPORTS) == set(_declared())


def test_library_holds_gfx950_code_only(lib_path):
    out = subprocess.run(["strings", lib_path], capture_output=True, text=True).stdout
    assert "gfx950" in out
    for other in ("gfx90a", "gfx942", "gfx1100", "sm_"):
        assert f"amdgcn-amd-amdhsa--{other}" not in out
