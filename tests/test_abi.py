"""The C-ABI library loads on the CPU host and exports every function that
include/kfbi.h declares (no device calls are made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2309_01068_amd", "libkfbi.so")


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for", "while", "return")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("kfbi_create", "kfbi_destroy", "kfbi_set_interface", "kfbi_apply",
                 "kfbi_operator", "kfbi_gmres_solve", "kfbi_last_error", "thetaL_create",
                 "thetaL_init", "thetaL_step", "thetaL_get_state", "thetaL_set_state",
                 "kfbi_apply_batch", "thetaL_size", "stefan_create", "stefan_init", "stefan_step",
                 "stefan_temperature", "stefan_thetal"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfbi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfbi.so not built")
def test_binding_export_list_matches_header():
    from paper_2309_01068_amd import kfbi
    assert set(kfbi.EXPORTS) <= set(declared_functions())
