"""CPU checks of the boundary: the HIP library loads and exports every entry
point that include/lbmib.h declares, and the binding knows each of them."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1803_09380_amd import lbmib
from paper_1803_09380_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmib.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("lbm_create", "ib_set_markers", "lbm_step", "ib_forces", "lbm_fields"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lbmib.LIB_PATH):
        pytest.fail("liblbmib.so is not built")
    lib = ctypes.CDLL(lbmib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    bound = {s[0] for s in lbmib.SIGNATURES}
    assert set(declared_functions()) == bound


def test_binding_struct_layouts():
    # lbm_params: 2 int32, 2 double, 5 int32 (+pad), 4 double, int32 (+pad),
    # 2 double, int32 (+pad), 9 double, int32 (+pad)
    assert ctypes.sizeof(lbmib.Params) == 192
    assert ctypes.sizeof(lbmib.Body) == 72


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, printed by a program that gcc
    builds against include/lbmib.h."""
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbmib.h"', "int main(void) {",
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct,cls", [("lbm_params", "Params"), ("ib_body", "Body")])
def test_binding_layout_matches_the_c_header(struct, cls, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    ct = getattr(lbmib, cls)
    names = [f[0] for f in ct._fields_]
    size, offs = _c_layout(struct, names, tmp_path)
    assert size == ctypes.sizeof(ct)
    assert offs == [getattr(ct, n).offset for n in names]


def test_version_string():
    assert lbmib.version().startswith("lbmib-gfx950")


def test_device_bytes_bound_is_host_arithmetic():
    """The bound needs no device: the population array of the row-blocked
    layout (rows -1 .. ny, blocks of 64 nodes with 9 populations, a ghost
    block and the x = nx ghost) plus a small IB term; invalid arguments give 0."""
    case = wl.settling(nx=400, ny=4000, D=40.0, density_ratio=1.2, two=True, lower=(200.0, 300.0))
    nblk = (400 + 64) // 64 + 1
    pop = nblk * 9 * 64 * (4000 + 2) * 4
    b32 = lbmib.device_bytes_bound(case, lbmib.F32_SHIFTED)
    assert pop < b32 < 1.01 * pop
    b64 = lbmib.device_bytes_bound(case, lbmib.F64)
    assert 2 * pop < b64 < 1.01 * 2 * pop
    L = lbmib.load()
    p = lbmib.make_params(64, 64, 0.8)
    counts = (ctypes.c_int32 * 9)(*([10] * 9))
    assert L.lbm_device_bytes_bound(None, 0, None) == 0
    assert L.lbm_device_bytes_bound(ctypes.byref(p), 9, counts) == 0
    assert L.lbm_device_bytes_bound(ctypes.byref(p), 1, None) == 0
    neg = (ctypes.c_int32 * 1)(-1)
    assert L.lbm_device_bytes_bound(ctypes.byref(p), 1, neg) == 0
    # more markers never lower the bound
    one = (ctypes.c_int32 * 1)(100)
    two = (ctypes.c_int32 * 1)(200)
    assert L.lbm_device_bytes_bound(ctypes.byref(p), 1, two) > L.lbm_device_bytes_bound(ctypes.byref(p), 1, one)
