"""The C-ABI library loads and exports every function its headers declare
(no compute calls: these run without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2110_14494_amd", "libpcmcc.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(pcmcc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_headers_declare_entry_points():
    names = declared_functions()
    for required in ("pcmcc_create", "pcmcc_init_species", "pcmcc_init_tables", "pcmcc_push_collide_deposit",
                     "pcmcc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_null_context_errors():
    lib = ctypes.CDLL(LIB)
    lib.pcmcc_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.pcmcc_version()
    lib.pcmcc_destroy.argtypes = [ctypes.c_void_p]
    assert lib.pcmcc_destroy(None) == 0
    lib.pcmcc_init_species.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4
    assert lib.pcmcc_init_species(None, 1.0, 1.0, 1.0, 1.0) == -1
