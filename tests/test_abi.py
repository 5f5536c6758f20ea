"""CPU checks of the C ABI: the library loads and exports every declared function,
and the pure host entry points validate their arguments (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(mg_[A-Za-z0-9_]+)\s*\(", src,
                            flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1410_8568_amd import mg
    L = mg.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/*.h but not exported"
    assert sorted(mg.EXPORTS) == sorted(names)


def test_workspace_bytes_and_validation():
    from paper_1410_8568_amd import mg
    o = mg.options()
    w32 = mg.workspace_bytes((32, 32, 32), o)
    w64 = mg.workspace_bytes((64, 64, 64), o)
    assert 40 * 32 ** 3 < w32 < 90 * 32 ** 3
    assert 7.0 < w64 / w32 < 9.0
    r = mg.options(precision="fp32_refined")
    assert mg.workspace_bytes((64, 64, 64), r) > w64 * 0.8
    for bad in [(1, 8, 8), (9, 9, 9), (0, 0, 0)]:
        with pytest.raises(mg.MGError) as ei:
            mg.workspace_bytes(bad, o)
        assert ei.value.status == mg.MG_E_INVALID
    o2 = mg.options(max_cycles=0)
    with pytest.raises(mg.MGError):
        mg.workspace_bytes((8, 8, 8), o2)


def test_status_strings_and_null_handles():
    from paper_1410_8568_amd import mg
    L = mg.lib()
    assert L.mg_status_string(mg.MG_OK) == b"MG_OK"
    assert b"BUDGET" in L.mg_status_string(mg.MG_E_BUDGET)
    assert L.mg_solve(None, None, None, ctypes.c_double(1e-10), None, None) == mg.MG_E_INVALID
    assert L.mg_level_dims(None, 0, None, None, None) == mg.MG_E_INVALID
    L.mg_destroy(None)
    L.mg_server_destroy(None)
    assert L.mg_default_options(None) == mg.MG_E_INVALID
