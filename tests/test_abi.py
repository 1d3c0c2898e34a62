"""The C ABI without a GPU: every function include/fr.h declares is exported
by libfr.so and bound by the Python layer, and the ctypes mirrors of the
argument structs have the C layout (checked against a C compiler)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2101_05356_amd import _lib  # noqa: E402

HEADER = os.path.join(ROOT, "include", "fr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(fr_\w+)\s*\(", text, flags=re.M))


@pytest.fixture(scope="module")
def libfr():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2101_05356_amd import build
        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_bound_functions():
    decl = declared_functions()
    assert len(decl) >= 25
    assert decl == set(_lib.exported_symbols())


def test_library_exports_every_declared_function(libfr):
    missing = [n for n in declared_functions() if not hasattr(libfr, n)]
    assert not missing, missing


def test_status_strings(libfr):
    f = libfr.fr_status_string
    f.restype = ctypes.c_char_p
    f.argtypes = [ctypes.c_int]
    texts = {f(i).decode() for i in range(9)}
    assert len(texts) == 9


STRUCTS = {"FrScene": "fr_scene", "FrRenderOpts": "fr_render_opts", "FrGrads": "fr_grads",
           "FrJobDesc": "fr_job_desc", "FrServerOpts": "fr_server_opts", "FrRequest": "fr_request",
           "FrResult": "fr_result", "FrStats": "fr_stats"}


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_struct_layout_matches_c(name, tmp_path):
    cname = STRUCTS[name]
    st = getattr(_lib, name)
    lines = [f'printf("%zu\\n", sizeof({cname}));']
    for fname, _t in st._fields_:
        lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fr.h\"\nint main(void){\n" +
                   "\n".join(lines) + "\nreturn 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(st)] + [getattr(st, f).offset for f, _ in st._fields_]
    assert got == want
