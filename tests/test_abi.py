"""libshg.so loads without a GPU and exports every entry point include/shg.h declares."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "shg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int64_t|int|void|const char \*)\s*\*?\s*(shg_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("shg_create", "shg_destroy", "shg_last_error", "shg_pairs", "shg_pairs_deriv", "shg_aab"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1701_06588_amd import shg
    lib = shg.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    for name in shg.EXPORTS:
        assert name in declared_functions(), name


def test_library_has_gfx950_code_object():
    from paper_1701_06588_amd import shg
    data = open(shg.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1701_06588_amd import shg
    with pytest.raises(RuntimeError):
        shg.Engine()
