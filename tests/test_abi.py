"""The C-ABI library without a GPU: it loads, exports every symbol include/evx.h declares, and
rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "evx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(evx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2507_21748_amd import evx
    return evx.load()


def test_header_declares_entry_points():
    names = _declared()
    for required in ("evx_plan_create", "evx_plan_destroy", "evx_ch_step", "evx_ch_begin",
                     "evx_ch_advance", "evx_ch_end", "evx_status_string", "evx_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    for s in range(8):
        assert lib.evx_status_string(s)
    assert lib.evx_status_string(99) == b"unknown status"


def test_nonfinite_status_and_params_layout(lib):
    """The failure check's status code and the params struct (check_finite after model) agree
    between the header, the library and the binding."""
    import re
    from paper_2507_21748_amd import evx
    text = open(HEADER).read()
    assert re.search(r"EVX_ERR_NONFINITE\s*=\s*7", text)
    assert b"non-finite" in lib.evx_status_string(7)
    body = re.search(r"typedef struct evx_ch_params \{(.*?)\} evx_ch_params;", text, re.S).group(1)
    fields = re.findall(r"(double|int)\s+(\w+);", body)
    assert [n for _, n in fields] == [n for n, _ in evx._Params._fields_]
    assert ctypes.sizeof(evx._Params) == 48


@pytest.mark.parametrize("nx,ny,nz,bc", [
    (14, 16, 16, 0),     # nx/2 = 7 not a supported length
    (33, 16, 16, 0),     # odd nx with periodic boundaries
    (16, 7, 16, 0),      # 7 not 2/3/5-smooth
    (16, 16, 2048, 1),   # beyond the largest length
    (18, 16, 16, 1),     # 18 not in the list (zero flux uses nx itself)
])
def test_plan_rejects_unsupported_sizes(lib, nx, ny, nz, bc):
    h = ctypes.c_void_p()
    st = lib.evx_plan_create(ctypes.byref(h), nx, ny, nz, bc, 0, 1.0)
    assert st == 2, lib.evx_last_error()
    assert h.value is None


@pytest.mark.parametrize("args", [
    (16, 16, 16, 5, 0, 1.0),     # bad bc
    (16, 16, 16, 0, 9, 1.0),     # bad scheme
    (16, 16, 16, 0, 0, 0.0),     # dx <= 0
    (0, 16, 16, 0, 0, 1.0),      # empty grid
    (16, -4, 16, 0, 0, 1.0),
])
def test_plan_rejects_bad_arguments(lib, args):
    h = ctypes.c_void_p()
    assert lib.evx_plan_create(ctypes.byref(h), *args) == 1
    assert lib.evx_last_error()


def test_null_arguments(lib):
    assert lib.evx_plan_create(None, 16, 16, 16, 0, 0, 1.0) == 1
    assert lib.evx_plan_destroy(None) == 1
    assert lib.evx_ch_step(None, None, 1, None, None) == 1
    assert lib.evx_ch_advance(None, 1, None, None) == 1


def test_params_struct_layout_matches_header(tmp_path):
    """The binding's evx_ch_params mirrors the C struct: size and every field offset, as the host
    compiler lays it out from include/evx.h."""
    import shutil
    import subprocess
    from paper_2507_21748_amd.evx import _Params
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "evx.h"\nint main(void) {\n'
                   '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(evx_ch_params),\n'
                   '         offsetof(evx_ch_params, dt), offsetof(evx_ch_params, M),\n'
                   '         offsetof(evx_ch_params, kappa), offsetof(evx_ch_params, A),\n'
                   '         offsetof(evx_ch_params, integrator),\n'
                   '         offsetof(evx_ch_params, model));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(_Params)] + [getattr(_Params, f).offset
                                       for f in ("dt", "M", "kappa", "A", "integrator", "model")]
    assert got == want
