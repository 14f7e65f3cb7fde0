"""The C ABI library loads, exports every entry point excmg.h declares, and rejects bad
arguments before touching the GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "excmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(excmg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1901_05118_amd as ex
    if not os.path.exists(ex.lib_path):
        from paper_1901_05118_amd import build
        build.build()
    return ex.load()


def test_header_declares_the_solver_entry_points():
    names = _declared()
    for required in ("excmg_solve", "excmg_apply_stencil", "excmg_setup", "excmg_finalize",
                     "excmg_last_error", "excmg_exp_finite", "excmg_exp_true", "excmg_rhs",
                     "excmg_bicg", "excmg_level_solve", "excmg_dsolve", "excmg_solve_ex"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_bad_arguments_are_rejected(lib):
    import paper_1901_05118_amd as ex
    c = ctypes.c_void_p(0)
    assert lib.excmg_setup(32, 4, 3) == ex.EINVAL          # bc kind
    assert lib.excmg_setup(32, 2, 1) == ex.EINVAL          # too few levels
    assert lib.excmg_setup(36, 4, 1) == ex.EINVAL          # not N0 * 2^(L-1)
    assert lib.excmg_setup(32 * 16, 4, 1) == ex.EINVAL     # coarsest grid too large
    assert "DSOLVE" in ex.last_error()
    assert lib.excmg_exp_finite(6, c, c, c) == ex.EINVAL
    assert lib.excmg_exp_true(7, c, c, c) == ex.EINVAL
    assert lib.excmg_apply_operator(1, 1, 0, c, c) == ex.EINVAL
    assert lib.excmg_apply_operator(8, 1, 0, None, None) == ex.EINVAL
    assert lib.excmg_apply_stencil(0, 0, c, c) == ex.ENOCTX  # no context
    assert "context" in ex.last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1901_05118_amd.excmg as mod
    monkeypatch.setattr(mod, "_lib", None)
    monkeypatch.setattr(mod, "lib_path", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        mod.load()


def test_binding_rejects_wrong_arrays():
    import numpy as np
    import paper_1901_05118_amd.excmg as mod
    with pytest.raises(TypeError):
        mod._ptr(np.zeros(4, dtype=np.float32))
    with pytest.raises(ValueError):
        mod._ptr(np.zeros(4), count=5)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of excmg_opts, excmg_level_stats, excmg_stats and excmg_problem
    have the header's sizes and field offsets (a C program compiled against excmg.h prints
    them)."""
    import shutil
    import subprocess

    from paper_1901_05118_amd import excmg as ex
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"excmg_opts": ex.Opts, "excmg_level_stats": ex.LevelStats,
               "excmg_stats": ex.Stats, "excmg_problem": ex.Problem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "excmg.h"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
