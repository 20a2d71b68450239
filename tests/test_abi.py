"""CPU checks of the library boundary: the shared library loads, exports
every entry point declared in include/lbm.h, and the binding's structures
match the header's layout.  No compute call is made (no GPU here)."""
import ctypes as C
import os
import re

import pytest

from paper_1503_06869_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libso():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1503_06869_amd import build
        build.build()
    return C.CDLL(lbm.LIB_PATH)


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ["lbm_create", "lbm_add_fiber", "lbm_step", "lbm_get_force_torque", "lbm_get_fields"]:
        assert n in names


def test_library_exports_every_declared_symbol(libso):
    missing = [n for n in declared_functions() if not hasattr(libso, n)]
    assert not missing, missing
    assert sorted(lbm.EXPORTED) == declared_functions()


def test_lattice_table_needs_no_gpu():
    c, w = lbm.lattice()
    assert c.shape == (19, 3) and abs(w.sum() - 1.0) < 1e-15
    for q in range(1, 19):
        assert any((c[p] == -c[q]).all() for p in range(19))


def test_struct_layout_matches_header():
    # lbm_params: 5 int32 (+4 pad), 4 doubles, 3 doubles, 4 int32, int64, pointer, 2 int32
    assert C.sizeof(lbm.lbm_params) == 5 * 4 + 4 + 4 * 8 + 3 * 8 + 4 * 4 + 8 + 8 + 2 * 4
    assert C.sizeof(lbm.lbm_fiber) == (3 + 4 + 3 + 3 + 3) * 8
    assert C.sizeof(lbm.lbm_info) == 8 + 4 + 4 + 8 * 4


def test_params_default_and_argument_errors(libso):
    L = lbm.load()
    p = lbm.lbm_params()
    assert L.lbm_params_default(C.byref(p)) == lbm.LBM_OK
    assert (p.nx, p.ny, p.nz) == (32, 32, 32) and p.tau == 0.8 and p.magic == 3.0 / 16.0
    h = C.c_void_p()
    bad = lbm.lbm_params()
    L.lbm_params_default(C.byref(bad))
    bad.tau = 0.5
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.tau, bad.wall_u = 0.8, 0.2
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    assert L.lbm_create(None, C.byref(h)) == lbm.LBM_E_ARG
    assert L.lbm_step(None, 1) == lbm.LBM_E_ARG
