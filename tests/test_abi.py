"""The C-ABI library loads on a GPU-less host and exports every entry point
include/pm.h declares (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1505_04694_amd import pmesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("pm.h", "pm3.h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pm3?_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_named_calls():
    names = declared()
    for n in ("pm_mesh_create", "pm_colour", "pm_coarsen", "pm_refine", "pm_swap", "pm_smooth", "pm_quality"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = pmesh.lib()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pmesh.EXPORTS) <= set(declared())
    from paper_1505_04694_amd import pmesh3
    assert set(pmesh3.EXPORTS3) <= set(declared())
    pmesh3.lib()  # every 3D entry point resolves


def test_options_layout_and_defaults():
    o = pmesh.pm_default_options()
    assert (o.L_low2, o.L_up2, o.q_min, o.slack) == (0.5, 2.0, 0.1, 2.0)
    assert (o.coarsen_rounds, o.swap_rounds, o.refine_passes, o.smooth_sweeps) == (200, 100, 32, 1)
    assert o.quality == pmesh.PM_QUALITY_MEAN_RATIO and o.reserved == 0
    assert ctypes.sizeof(pmesh.Options) == 128
    assert not o.allocator
    assert ctypes.sizeof(pmesh.Tuning) == 32
    assert ctypes.sizeof(pmesh.Context) == 24
    assert ctypes.sizeof(pmesh.Stats) == 128


def test_binding_structs_match_the_header(tmp_path):
    """sizeof and field offsets of the header's structs, compiled with the
    host C compiler, equal those of the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_1505_04694_amd import pmesh3
    structs = {"pm_options": pmesh.Options, "pm_tuning": pmesh.Tuning, "pm_context": pmesh.Context,
               "pm3_mesh_desc": pmesh3.MeshDesc3,
               "pm_stats": pmesh.Stats, "pm_mesh_desc": pmesh.MeshDesc, "pm_allocator": pmesh.Allocator}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pm3.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def test_argument_errors_without_gpu():
    lib = pmesh.lib()
    # an unknown quality functional is refused before any device work
    o = pmesh.pm_default_options(quality=5)
    xy = np.array([[0, 0], [1, 0], [0, 1]], float)
    tri = np.array([[0, 1, 2]], np.int32)
    met = np.tile([1.0, 0.0, 1.0], (3, 1))
    d = pmesh.MeshDesc(xy.ctypes.data, tri.ctypes.data, met.ctypes.data, None, 3, 1, pmesh.PM_MEM_HOST)
    h = ctypes.c_void_p()
    assert lib.pm_mesh_create(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h)) == pmesh.PM_E_ARG
    assert lib.pm_default_options(None) == pmesh.PM_E_ARG
    assert lib.pm_mesh_create(None, None, None, None) == pmesh.PM_E_ARG
    assert lib.pm_mesh_destroy(None) == pmesh.PM_OK
    assert lib.pm_last_error(None) in (b"null handle", b"pm_mesh_create failed")


def test_tetrahedral_argument_errors_without_gpu():
    from paper_1505_04694_amd import pmesh3
    lib = pmesh3.lib()
    h = ctypes.c_void_p()
    assert lib.pm3_mesh_create(None, None, None, ctypes.byref(h)) == pmesh.PM_E_ARG
    xyz = np.zeros((3, 3))
    tet = np.array([[0, 1, 2, 0]], np.int32)
    met = np.tile([1.0, 0, 0, 1.0, 0, 1.0], (3, 1))
    d = pmesh3.MeshDesc3(xyz.ctypes.data, tet.ctypes.data, met.ctypes.data, None, 3, 1, pmesh.PM_MEM_HOST)
    assert lib.pm3_mesh_create(ctypes.byref(d), None, None, ctypes.byref(h)) == pmesh.PM_E_ARG   # V < 4
    d = pmesh3.MeshDesc3(xyz.ctypes.data, tet.ctypes.data, met.ctypes.data, None, 4, 0, pmesh.PM_MEM_HOST)
    assert lib.pm3_mesh_create(ctypes.byref(d), None, None, ctypes.byref(h)) == pmesh.PM_E_ARG   # no element
    assert lib.pm3_mesh_destroy(None) == pmesh.PM_OK
    assert lib.pm3_mesh_sizes(None, None, None) == pmesh.PM_E_ARG
