"""The C-ABI library loads and exports every entry point include/adjoint.h
declares (no compute calls: this runs on the CPU)."""

import ctypes
import os
import re

from conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "adjoint.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:adj_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def _lib_path():
    from paper_2603_16478_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2603_16478_amd import build
        build.build()
    return native.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("adj_scene_create", "adjoint_setup", "adjoint_solve", "vjp_params", "sim_forward_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2603_16478_amd import native
    assert sorted(native.EXPORTS) == _declared()
