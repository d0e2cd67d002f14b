"""The C ABI without a GPU: the library loads, exports every entry point that
include/vfpi.h declares, and rejects bad arguments synchronously before any
device work."""
import ctypes
import os
import re

import pytest

import paper_2201_09212_amd as vf
from paper_2201_09212_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vfpi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(vfpi_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_entry_points():
    assert _declared() == sorted(_abi.ENTRY_POINTS)


def test_library_exports_every_declared_symbol():
    lib = vf.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_error_strings():
    for code in range(-7, 1):
        assert vf.vfpi_error_string(code) != "unknown error code"
    assert vf.vfpi_error_string(-99) == "unknown error code"


def test_tape_bytes():
    assert vf.vfpi_tape_bytes(0, 0) == 0
    assert vf.vfpi_tape_bytes(100, 100) == 7680  # 48*100 + 28*100 = 7600 -> 256-aligned
    assert vf.vfpi_tape_bytes(1, 0) == 256
    assert vf.vfpi_tape_bytes(-1, 0) == _abi.VFPI_E_SHAPE


def test_null_and_shape_errors_before_device_work():
    lib = vf.load()
    A = _abi.vfpi_bsr(4, 4, None, None, None)
    Jc = _abi.vfpi_contacts(0, 0, None, None, None, None, None)
    o = vf.make_opts()
    assert lib.vfpi_step(None, ctypes.byref(A), None, ctypes.byref(Jc), None, None, ctypes.byref(o), None, None,
                         None) == _abi.VFPI_E_NULL
    assert lib.vfpi_step_batched(None, 1, None, None, None, ctypes.byref(A), None, ctypes.byref(Jc), None, None,
                                 ctypes.byref(o), None, None) == _abi.VFPI_E_NULL
    assert lib.vfpi_step_backward(None, ctypes.byref(A), ctypes.byref(Jc), None, None, None, None, None, None,
                                  None, None, ctypes.byref(o), None, None) == _abi.VFPI_E_NULL
    assert lib.vfpi_create(None, 1, 1, 1, 0) == _abi.VFPI_E_NULL
    h = ctypes.c_void_p()
    assert lib.vfpi_create(ctypes.byref(h), -1, 1, 1, 0) == _abi.VFPI_E_SHAPE
    assert h.value is None
    assert lib.vfpi_destroy(None) == _abi.VFPI_OK


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        _abi._lib_saved = _abi._lib
        try:
            _abi._lib = None
            _abi.load(str(tmp_path / "nope.so"))
        finally:
            _abi._lib = _abi._lib_saved


def test_header_layout_matches_binding(tmp_path):
    """The descriptor structs as a C compiler lays them out from the header:
    every field's offset and every struct's size equal the Python binding's
    (a C program that only includes the header; nothing runs on a GPU)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    hip_inc = "/opt/rocm/include"
    if gcc is None or not os.path.isdir(hip_inc):
        pytest.skip("needs gcc and the HIP headers")
    structs = [_abi.vfpi_bsr, _abi.vfpi_contacts, _abi.vfpi_opts, _abi.vfpi_stats]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "vfpi.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append(f'  printf("{n} sizeof %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-D__HIP_PLATFORM_AMD__", f"-I{os.path.join(ROOT, 'include')}",
                    f"-I{hip_inc}", str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for st in structs:
        n = st.__name__
        assert got[(n, "sizeof")] == ctypes.sizeof(st), n
        for f, _ in st._fields_:
            assert got[(n, f)] == getattr(st, f).offset, (n, f)
