"""The C-ABI library loads and exports every function declared in
include/mrcm.h (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrcm.h")
LIB = os.path.join(ROOT, "paper_2404_13811_amd", "libmrcm.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:mrcm_status|const char\*)\s+(mrcm_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_paper_shaped_calls():
    names = declared()
    for n in ("mrcm_create", "mrcm_set_permeability", "mrcm_set_partition", "mrcm_set_interface_space",
              "mrcm_set_robin", "mrcm_build_basis", "mrcm_solve_interface", "mrcm_smooth",
              "mrcm_get_pressure", "mrcm_get_flux", "mrcm_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_the_abi():
    import paper_2404_13811_amd as m
    for n in declared():
        short = n[len("mrcm_"):]
        if short in ("last_error",):
            continue
        assert hasattr(m, short), short
