"""CPU checks of the boundary: the HIP library loads and exports every entry
point that include/lbmib.h declares, and the binding knows each of them."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1803_09380_amd import lbmib

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
