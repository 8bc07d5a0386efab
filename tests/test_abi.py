"""The C ABI library loads without a GPU and exports every function that
include/wdsolve.h declares; the Python binding declares the same set."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdsolve.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \t\*]*?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    import paper_0907_3261_amd as pkg
    from paper_0907_3261_amd import build as b
    if not os.path.exists(pkg.LIB_PATH):
        b.build()
    return pkg.load()


def test_header_parses():
    names = header_functions()
    for must in ("wd_create", "wd_apply", "jacobi_precond", "bbicggr_solve", "wd_block_gram"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_0907_3261_amd._binding import SIGNATURES
    bound = sorted(n for n, _, _ in SIGNATURES)
    assert bound == header_functions()


def test_strerror_without_gpu(lib):
    import paper_0907_3261_amd as pkg
    assert pkg.strerror(0) == "ok"
    assert "invalid" in pkg.strerror(-1)
    assert "breakdown" in pkg.strerror(2)


def test_argument_checks_without_gpu(lib):
    """Entry points reject bad arguments before any HIP call, so this runs on the CPU."""
    import ctypes
    from ctypes import c_int, c_void_p
    import paper_0907_3261_amd as pkg
    L = pkg.load()                                    # argument and result types set from the header table
    h = c_void_p()

    def create(dims, bc_t=0, max_L=4):
        return L.wd_create(ctypes.byref(h), (c_int * 4)(*dims), bc_t, max_L, None)

    assert create((4, 4, 1, 4)) == -1                 # extent below 2
    assert create((4, 4, 4, 4), bc_t=2) == -1         # boundary flag
    assert create((4, 4, 4, 4), max_L=0) == -1
    assert create((4, 4, 4, 4), max_L=pkg.WD_MAX_L + 1) == -1
    assert create((1024, 1024, 512, 2)) == -1          # 2^29 sites: above the 2^28 limit
    assert not h.value
    assert L.wd_create(None, (c_int * 4)(4, 4, 4, 4), 0, 4, None) == -1
    assert L.wd_destroy(None) == -1
    info = pkg._binding.SolveInfo()
    info.status = 123
    for solve in (L.bbicggr_solve, L.bbicgstab_solve):
        assert solve(None, None, None, 4, 1e-12, None, ctypes.byref(info)) == -1
    assert info.status == 123                         # argument errors leave info untouched


def test_header_is_plain_c99_and_links(tmp_path, lib):
    """The ABI header compiles as strict C99, and a C program links against the library
    and gets WD_EINVAL for a bad extent without touching the GPU."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "abi.c"
    src.write_text(
        '#include <stdio.h>\n#include "wdsolve.h"\n'
        "int main(void) {\n"
        "    wd_ctx* c = 0;\n"
        "    const int dims[4] = {4, 4, 1, 4};\n"
        "    int r = wd_create(&c, dims, 0, 4, 0);\n"
        '    printf("%d %s\\n", r, wd_strerror(r));\n'
        "    return (r == WD_EINVAL && c == 0) ? 0 : 1;\n"
        "}\n")
    import paper_0907_3261_amd as pkg
    exe = tmp_path / "abi"
    libdir = os.path.dirname(pkg.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.dirname(HEADER), str(src),
           "-o", str(exe), "-L", libdir, "-lwdsolve", "-Wl,-rpath," + libdir]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "invalid argument" in out.stdout


def test_struct_layouts_match_header():
    """Field order and sizes of the option/info structs mirror the C declarations."""
    import ctypes
    from paper_0907_3261_amd._binding import SolveInfo, SolveOpts
    text = open(HEADER).read()
    for struct, cls in (("wd_solve_opts", SolveOpts), ("wd_solve_info", SolveInfo)):
        body = re.search(r"typedef struct %s \{(.*?)\}" % struct, text, flags=re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(\w+)(?:\[\w+\])?\s*;", body)
        assert fields == [f for f, _ in cls._fields_]
    assert ctypes.sizeof(SolveInfo) == 7 * 4 + 4 + 8 * 2 + 8 + 8 + 2 * 16 * 8 + 8 + 2 * 4


def test_binding_constants_match_header():
    """Every #define of the header that the binding also names has the same value there."""
    from paper_0907_3261_amd import _binding as b
    text = open(HEADER).read()
    defines = dict(re.findall(r"^#define (WD_\w+)\s+\(?(-?\d+)\)?", text, flags=re.M))
    shared = [n for n in defines if hasattr(b, n)]
    for must in ("WD_F64", "WD_F32", "WD_BF16", "WD_F64_COEF_F32", "WD_F64_COEF_BF16", "WD_MAX_L",
                 "WD_PRECOND_LEARNED", "WD_EINVAL", "WD_STAGNATED"):
        assert must in shared, must
    for n in shared:
        assert getattr(b, n) == int(defines[n]), n
    # the precision names of the binding map onto header constants
    assert set(b.PREC.values()) == {int(defines[n]) for n in
                                    ("WD_F64", "WD_F32", "WD_BF16", "WD_F64_COEF_F32", "WD_F64_COEF_BF16")}
