"""CPU checks of the boundary: the HIP library loads and exports every
symbol that include/sdem.h declares (no compute calls; no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "sdem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdem_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("sdem_init", "sdem_add_mesh", "sdem_step", "sdem_read_state"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2507_12610_amd import sdem
    if not os.path.exists(sdem.LIB_PATH):
        pytest.skip("libsdem.so not built")
    lib = ctypes.CDLL(sdem.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(sdem.EXPORTS) == set(declared_symbols())


def test_workspace_bytes_and_config_checks():
    """Pure host arithmetic of the ABI: sizes grow with capacities and bad
    configurations are rejected (returns 0)."""
    from paper_2507_12610_amd import sdem
    if not os.path.exists(sdem.LIB_PATH):
        pytest.skip("libsdem.so not built")
    L = sdem.lib()
    c1 = sdem.Config(1000, 8000, 10000, 12, 1, 0, 0, 0, 1.0)
    c2 = sdem.Config(2000, 8000, 10000, 12, 1, 0, 0, 0, 1.0)
    b1 = L.sdem_workspace_bytes(ctypes.byref(c1))
    b2 = L.sdem_workspace_bytes(ctypes.byref(c2))
    assert 0 < b1 < b2
    assert b1 % 256 == 0
    for bad in (sdem.Config(-1, 8000, 10000, 12, 1, 0, 0, 0, 1.0),
                sdem.Config(1000, 8000, 0, 12, 1, 0, 0, 0, 1.0),
                sdem.Config(1000, 8000, 10000, 12, 0, 0, 0, 0, 1.0),
                sdem.Config(1000, 8000, 10000, 12, 1, 7, 0, 0, 1.0),
                sdem.Config(1000, 8000, 10000, 12, 1, 0, 65, 0, 1.0),
                sdem.Config(1000, 8000, 10000, 12, 1, 0, 0, 0, 1.0, -1.0),
                sdem.Config(1000, 8000, 10000, 12, 1, 0, 0, 0, 0.1)):
        assert L.sdem_workspace_bytes(ctypes.byref(bad)) == 0
    assert b"cell_factor" in L.sdem_last_error()
    assert L.sdem_workspace_bytes(ctypes.byref(sdem.Config(1000, 8000, 10000, 12, 1, 0, 0, 0, 1.0,
                                                           -1.0))) == 0
    assert b"skin" in L.sdem_last_error()
