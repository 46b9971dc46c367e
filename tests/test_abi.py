"""The C-ABI library loads and exports every entry point declared in include/tdbem.h (no GPU needed)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tdbem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdbem_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    from paper_2111_05205_amd import _native
    L = _native.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_invalid_meshes_rejected_before_device_work():
    import synth
    from paper_2111_05205_amd import _native as N
    L = N.lib()
    xyz, tri = synth.icosphere(1)

    def create(v, f, c=1.0, dt=0.1, d=1):
        v = np.ascontiguousarray(v, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.int32)
        m = N.Mesh(v.shape[0], f.shape[0], v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        h = ctypes.c_void_p()
        rc = L.tdbem_create(ctypes.byref(m), c, dt, d, 1, 0, None, None, ctypes.byref(h))
        return rc, L.tdbem_last_error(None).decode()

    assert create(xyz, tri[:-1])[0] == N.E_INVAL                      # open surface
    bad = tri.copy(); bad[0] = bad[0][[0, 2, 1]]
    assert create(xyz, bad)[0] == N.E_INVAL                           # inconsistent orientation
    bad = tri.copy(); bad[3, 1] = 10 ** 6
    assert create(xyz, bad)[0] == N.E_INVAL                           # index out of range
    assert create(xyz, tri, c=-1.0)[0] == N.E_INVAL
    assert create(xyz, tri, d=4)[0] == N.E_INVAL
    assert create(xyz, tri, dt=0.0)[0] == N.E_INVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import importlib
    from paper_2111_05205_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    try:
        _native.lib()
    except RuntimeError as e:
        assert "missing" in str(e)
    else:
        raise AssertionError("expected a RuntimeError")


def test_header_is_plain_c_and_links(tmp_path):
    """include/tdbem.h compiles as C99 with warnings as errors, and a C program links
    libtdbem.so and calls it (argument checks only; no device work)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        import pytest
        pytest.skip("no C compiler")
    from paper_2111_05205_amd import _native
    lib = os.path.abspath(_native.LIB_PATH)
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "tdbem.h"
int main(void) {
  tdbem_mesh m;
  struct tdbem_ctx *ctx = 0;
  memset(&m, 0, sizeof m);
  int rc = tdbem_create(&m, 1.0, 0.1, 2, TDBEM_BMBIE, TDBEM_NEUMANN, NULL, NULL, &ctx);
  printf("%d %s\n", rc, tdbem_last_error(NULL));
  rc = tdbem_create(&m, 1.0, 0.1, 2, TDBEM_BMBIE, TDBEM_NEUMANN, NULL, NULL, NULL);
  printf("%d\n", rc);
  tdbem_destroy(NULL);
  return ctx != 0;
}
''')
    exe = tmp_path / "use"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", inc, str(src), lib,
                    "-Wl,-rpath," + os.path.dirname(lib), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.splitlines()
    assert lines[0].startswith(str(_native.E_INVAL) + " ") and "NULL" in lines[0]
    assert lines[1] == str(_native.E_INVAL)


def test_binding_signatures_match_the_header():
    """Every ctypes declaration in the binding has the header's parameter count, with a
    pointer exactly where the prototype has one (a missing or integer-typed pointer
    argument would truncate addresses)."""
    from paper_2111_05205_amd import _native
    L = _native.lib()
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "tdbem.h")).read(), flags=re.S)
    protos = re.findall(r"\b(tdbem_[a-z_]+)\s*\(([^)]*)\)\s*;", src)
    assert len(protos) == len(_declared())

    def is_ptr(t):
        return t in (ctypes.c_void_p, ctypes.c_char_p) or (isinstance(t, type) and issubclass(t, ctypes._Pointer))
    for name, params in protos:
        params = params.strip()
        ps = [] if params in ("", "void") else [p.strip() for p in params.split(",")]
        at = getattr(L, name).argtypes
        assert at is not None, name
        assert len(at) == len(ps), name
        assert ["*" in p for p in ps] == [is_ptr(t) for t in at], name


def test_binding_structs_match_the_header_layout(tmp_path):
    """Size and field offsets of every struct the binding mirrors, as the C compiler lays
    them out from include/tdbem.h (a field added on one side only shifts the rest)."""
    import shutil
    import subprocess
    import pytest
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2111_05205_amd import _native as N
    pairs = [("tdbem_mesh", N.Mesh), ("tdbem_opts", N.Opts), ("tdbem_incident", N.Incident),
             ("tdbem_step_info", N.StepInfo), ("tdbem_run_info", N.RunInfo), ("tdbem_info", N.Info)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tdbem.h"', "int main(void) {"]
    want = []
    for cname, cls in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fname}));')
            want.append(getattr(cls, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == want
