"""The C ABI library loads and exports every entry point include/ccg.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
HEADER = os.path.join(ROOT, "include", "ccg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ccg_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("ccg_create", "ccg_destroy", "ccg_last_error", "ccg_solve", "ccg_debug_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (load torch's HIP runtime first, as the binding does)
    from paper_1204_0069_amd import LIB_PATH, EXPORTS
    assert os.path.exists(LIB_PATH), "libccg.so not built"
    lib = ctypes.CDLL(LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(EXPORTS) == sorted(declared_functions())


def test_binding_loads_without_gpu():
    from paper_1204_0069_amd import load_library
    lib = load_library()
    assert lib.ccg_last_error(None) == b"null context"


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_1204_0069_amd import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.ccg_create(ctypes.byref(h), 0, 0, None)
    assert st == -6 and not h.value
