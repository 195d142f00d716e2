"""The C-ABI library loads and exports every function include/md.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")
LIB = os.path.join(ROOT, "paper_2405_07898_amd", "libmdeam.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:md_status|void|const char\*)\s+(md_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("md_create", "md_build_neighbors", "md_step", "md_energy", "md_fm_forward",
                     "md_fm_backward", "md_autotune"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_binding_matches_header():
    from paper_2405_07898_amd import md

    assert sorted(md.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.md_status_string.restype = ctypes.c_char_p
    assert lib.md_status_string(0) == b"ok"
    assert b"capacity" in lib.md_status_string(-4)
