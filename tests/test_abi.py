"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point declared in include/sph.h, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")
LIB = os.path.join(ROOT, "paper_2603_19764_amd", "libsph.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("sph_build_cells", "sph_density", "sph_gradients", "sph_forces_stress",
                     "sph_stress_update"):
        assert required in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsph.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_context_and_bad_create_arguments(lib):
    lib.sph_build_cells.restype = C.c_int
    assert lib.sph_build_cells(None, C.c_int64(0), None, None, None, None, 1, None,
                               C.c_double(0.0), None, None) == 1  # SPH_EINVAL
    lib.sph_density.restype = C.c_int
    assert lib.sph_density(None, C.c_int64(0), *([None] * 18)) == 1
    out = C.c_void_p()
    lib.sph_create.restype = C.c_int
    lib.sph_create.argtypes = [C.POINTER(C.c_void_p), C.c_int64, C.c_int32, C.c_int64, C.c_int32,
                               C.c_int32]
    assert lib.sph_create(C.byref(out), 0, 64, 1 << 20, 1, 0) == 1       # capacity 0
    assert lib.sph_create(C.byref(out), 1 << 27, 64, 1 << 20, 1, 0) == 1  # above 2^26
    assert lib.sph_create(C.byref(out), 100, 0, 1 << 20, 1, 0) == 1       # no neighbours
    assert lib.sph_create(None, 100, 64, 1 << 20, 1, 0) == 1
    lib.sph_last_error.restype = C.c_char_p
    assert lib.sph_last_error(None) == b"null context"


def declared_arity():
    """Number of parameters of every function declared in the header."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(sph_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_the_header():
    """Every entry point the Python binding declares takes as many arguments
    as the header gives it (a missing one would shift the stream handle)."""
    from paper_2603_19764_amd import sph
    L = sph.lib()
    arity = declared_arity()
    checked = 0
    for name, n in arity.items():
        f = getattr(L, name)
        if f.argtypes is None:
            continue
        assert len(f.argtypes) == n, (name, len(f.argtypes), n)
        checked += 1
    assert checked >= 25


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2603_19764_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "liboracle", "sph_oracle"):
                    assert bad not in text, (f, bad)
