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


def test_scene_create_rejects_too_many_contacts_before_any_device_work():
    # the dense capacitance inverse of one scene is capped at 10000 contacts;
    # the argument check runs before the scene is built or the device touched
    lib = ctypes.CDLL(_lib_path())
    from paper_2603_16478_amd import native
    handle = ctypes.c_void_p()
    st = lib.adj_scene_create(ctypes.byref(native.SceneDesc()), ctypes.c_int32(10001), ctypes.byref(handle))
    assert native.STATUS[st] == "ADJ_E_ARG" and not handle.value
    lib.adj_last_error.restype = ctypes.c_char_p
    assert b"10000" in lib.adj_last_error()


def test_binding_declares_argument_types_of_every_entry_point():
    # an undeclared ctypes signature passes Python ints as 32-bit C ints,
    # which truncates device pointers
    from paper_2603_16478_amd import native
    lib = native.load()
    missing = [n for n in native.EXPORTS if n != "adj_last_error" and getattr(lib, n).argtypes is None]
    assert not missing, missing


def test_enum_values_agree_with_the_binding():
    """The enumerators of include/adjoint.h and the constants of the Python
    binding (the two sides of the ABI) carry the same values."""
    from paper_2603_16478_amd import native
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "adjoint.h")).read(), flags=re.S)
    enums = {}
    for body in re.findall(r"typedef enum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"(\w+)\s*=\s*(-?\d+)", body):
            enums[name] = int(val)
    pairs = {"ADJ_FP64": native.ADJ_FP64, "ADJ_MIXED": native.ADJ_MIXED, "ADJ_AUTO": native.ADJ_AUTO,
             "ADJ_GMRES": native.ADJ_GMRES, "ADJ_PCG": native.ADJ_PCG, "ADJ_SEMI_IMPLICIT": native.ADJ_SEMI_IMPLICIT,
             "ADJ_PRECOND_WOODBURY": native.PRECOND_WOODBURY,
             "ADJ_PRECOND_SPARSE_INVERSE": native.PRECOND_SPARSE_INVERSE,
             "ADJ_PRECOND_JACOBI": native.PRECOND_JACOBI, "ADJ_PRECOND_POINT_JACOBI": native.PRECOND_POINT_JACOBI,
             "ADJ_PRECOND_WOODBURY_NO_Z": native.PRECOND_WOODBURY_NO_Z,
             "ADJ_MAT_NEO_HOOKEAN": native.MAT_NEO_HOOKEAN, "ADJ_MAT_ARAP": native.MAT_ARAP,
             "ADJ_MAT_COROT": native.MAT_COROT}
    for name, val in pairs.items():
        assert enums[name] == val, name
    for code, name in native.STATUS.items():
        assert enums[name] == code, name


def test_struct_layouts_agree_with_the_header(tmp_path):
    """Size and field offsets of every struct of include/adjoint.h, as a C
    compiler lays them out, equal those of the binding's ctypes mirrors."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        import pytest
        pytest.skip("no C compiler")
    from paper_2603_16478_amd import native
    mirrors = {"adj_scene_desc": native.SceneDesc, "adj_contact_state": native.ContactState,
               "adj_solve_opts": native.SolveOpts, "adj_solve_info": native.SolveInfo, "adj_tuning": native.Tuning,
               "adj_batch_tuning": native.BatchTuning}
    # fields the binding names differently (a Python keyword in C)
    cfield = {("adj_contact_state", "lam"): "lambda"}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "adjoint.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = cfield.get((cname, fname), fname)
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
