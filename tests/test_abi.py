"""CPU checks of the C ABI boundary: the library loads and exports every entry
point include/regdock.h declares (no device calls)."""
import ctypes
import os
import re

import paper_2605_21398_amd as rd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "regdock.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+\**(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("register_init", "score_rotations", "register_free", "register_last_error"):
        assert n in names
    assert sorted(rd.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rd.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_loads_without_device():
    L = rd.load_library()
    assert L.register_last_error() is not None
