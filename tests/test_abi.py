"""CPU checks of the library boundary: the shared library loads, exports
every entry point declared in include/*.h, and the binding's structures
match the headers' layout.  No compute call is made (no GPU here)."""
import ctypes as C
import os
import re

import pytest

from paper_1503_06869_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header=None):
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in ([header] if header else sorted(os.listdir(inc))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(inc, h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b((?:lbm|sbf)_[a-z_]+)\s*\(", src))
    return sorted(names)


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
    assert sorted(lbm.EXPORTED) == declared_functions("lbm.h")
    assert sorted(lbm.EXPORTED_BATCH) == declared_functions("lbm_batch.h")
    assert sorted(lbm.EXPORTED_MLP) == declared_functions("lbm_mlp.h")
    from paper_1503_06869_amd import sbf
    assert sorted(sbf.EXPORTED_SBF) == declared_functions("sbf.h")


def test_lattice_table_needs_no_gpu():
    c, w = lbm.lattice()
    assert c.shape == (19, 3) and abs(w.sum() - 1.0) < 1e-15
    for q in range(1, 19):
        assert any((c[p] == -c[q]).all() for p in range(19))


def test_struct_layout_matches_header():
    # lbm_params: 5 int32 (+4 pad), 4 doubles, 3 doubles, 4 int32, int64, pointer, 4 int32, 2 doubles, 2 int32
    assert C.sizeof(lbm.lbm_params) == 5 * 4 + 4 + 4 * 8 + 3 * 8 + 4 * 4 + 8 + 8 + 4 * 4 + 2 * 8 + 2 * 4
    # centre, quaternion, L, r, density ratio, V, W; shape + reserved; force, torque
    assert C.sizeof(lbm.lbm_fiber) == (3 + 4 + 3 + 3 + 3) * 8 + 2 * 4 + 6 * 8
    assert C.sizeof(lbm.lbm_info) == 8 + 4 + 4 + 8 * 4
    # lbm_batch_case: 3 int32 (+4 pad), 2 doubles, lbm_fiber
    assert C.sizeof(lbm.lbm_batch_case) == 3 * 4 + 4 + 2 * 8 + C.sizeof(lbm.lbm_fiber)
    # lbm_batch_params: int32 (+4), 2 doubles, 4 int32, int64, pointer, 2 int32
    assert C.sizeof(lbm.lbm_batch_params) == 4 + 4 + 2 * 8 + 4 * 4 + 8 + 8 + 2 * 4
    assert C.sizeof(lbm.lbm_batch_tuning) == 4 + 4 + 8 + 4 + 4
    assert C.sizeof(lbm.lbm_batch_info) == 8 + 4 * 3 + 4 + 8 * 4


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
    bad.wall_u, bad.stabilize = 0.0, 2
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.stabilize, bad.contact_stiffness, bad.contact_range = 0, 1.0, 0.0
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.contact_stiffness = -1.0
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.contact_stiffness, bad.x_walls = 0.0, 3
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.x_walls, bad.y_walls = 0, -1
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    # free-slip z walls need non-periodic z and resting walls
    bad.y_walls, bad.z_free_slip, bad.z_periodic = 0, 1, 1
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.z_periodic, bad.wall_u = 0, 0.01
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    bad.wall_u, bad.z_free_slip = 0.0, 2
    assert L.lbm_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG
    assert L.lbm_step(None, 1) == lbm.LBM_E_ARG


def test_batch_argument_errors(libso):
    """Invalid batch arguments are rejected before any device call."""
    L = lbm.load()
    p = lbm.lbm_batch_params()
    assert L.lbm_batch_params_default(C.byref(p)) == lbm.LBM_OK
    assert p.storage == lbm.LBM_F32 and p.init_profile == lbm.LBM_INIT_COUETTE
    h = C.c_void_p()
    arr = (lbm.lbm_batch_case * 1)()
    arr[0].nx = arr[0].ny = arr[0].nz = 32
    arr[0].tau, arr[0].wall_u = 0.8, 0.005
    arr[0].fiber = lbm._fiber_struct((15.5, 15.5, 15.5), (1, 0, 0, 0), 16.0, 2.0)
    assert L.lbm_batch_create(C.byref(p), arr, 0, C.byref(h)) == lbm.LBM_E_ARG
    bad = lbm.lbm_batch_params()
    L.lbm_batch_params_default(C.byref(bad))
    bad.threads = 300
    assert L.lbm_batch_create(C.byref(bad), arr, 1, C.byref(h)) == lbm.LBM_E_ARG
    arr[0].tau = 0.5
    assert L.lbm_batch_create(C.byref(p), arr, 1, C.byref(h)) == lbm.LBM_E_GEOM
    assert b"case 0" in L.lbm_batch_last_error(None)
    arr[0].tau = 0.8
    arr[0].fiber = lbm._fiber_struct((15.5, 15.5, 15.5), (1, 0, 0, 0), 30.0, 2.0)
    assert L.lbm_batch_create(C.byref(p), arr, 1, C.byref(h)) == lbm.LBM_E_GEOM
    assert L.lbm_batch_step(None, 1) == lbm.LBM_E_ARG


def test_checkpoint_load_rejects_missing_and_foreign_files(libso, tmp_path):
    """lbm_load refuses a missing file and a file without the checkpoint
    header before touching the device, and returns no context."""
    L = lbm.load()
    h = C.c_void_p(123)
    assert L.lbm_load(str(tmp_path / "none.ckpt").encode(), None, C.byref(h)) == lbm.LBM_E_ARG
    assert not h.value
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint at all" * 4)
    h = C.c_void_p(123)
    assert L.lbm_load(str(bad).encode(), None, C.byref(h)) == lbm.LBM_E_ARG
    assert not h.value



def test_sbf_struct_layout_and_argument_errors(libso):
    """sbf_params matches the header (5 int32 + 1 reserved, 4 doubles, a
    pointer); invalid parameters are rejected before any device call."""
    from paper_1503_06869_amd import sbf
    assert C.sizeof(sbf.sbf_params) == 6 * 4 + 4 * 8 + 8
    L = sbf._lib()
    p = sbf.sbf_params()
    assert L.sbf_params_default(C.byref(p)) == lbm.LBM_OK
    assert (p.nmodes, p.nq, p.gmres_restart) == (5, 16, 30)
    h = C.c_void_p()
    for field, value in (("nmodes", 9), ("nq", 0), ("gmres_restart", 64), ("eps", 0.5), ("length", 0.0)):
        bad = sbf.sbf_params()
        L.sbf_params_default(C.byref(bad))
        setattr(bad, field, value)
        assert L.sbf_create(C.byref(bad), C.byref(h)) == lbm.LBM_E_ARG, field
    assert L.sbf_solve(None) == lbm.LBM_E_ARG
