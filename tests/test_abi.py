"""CPU checks of the C-ABI library: it builds, loads and exports every
function include/dem.h declares (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2106_09576_amd import build
    if not os.path.exists(build.library_path()):
        build.build()
    return build.library_path()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dem_create", "dem_set_particles", "dem_add_planar_wall",
                     "dem_add_cylinder_wall", "dem_step", "dem_get_state", "dem_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(lib_path):
    from paper_2106_09576_amd.dem import SIGNATURES, load_library
    assert set(SIGNATURES) == set(declared_functions())
    load_library()


def test_library_is_gfx950_code_object(lib_path):
    data = open(lib_path, "rb").read()
    assert b"gfx950" in data


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2106_09576_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|liboracle|oracle_dem)", text), f
