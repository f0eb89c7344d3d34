"""CPU-side checks of the C-ABI boundary: the library loads, exports every entry
point declared in include/phisft_sim.h, and the binding refuses to run without it."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phisft_sim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sim_create", "sim_create_batch", "sim_rollout", "sim_adjoint", "sim_sync_status",
              "sim_get_stats", "sim_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2203_11938_amd import sim
    if not os.path.exists(sim.LIB_PATH):
        pytest.fail("libphisft_sim.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(sim.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sim.EXPORTS)


def test_status_strings_without_gpu():
    from paper_2203_11938_amd import sim
    lib = sim.load_library()
    assert lib.sim_status_string(sim.SIM_OK) == b"ok"
    assert b"converge" in lib.sim_status_string(sim.SIM_E_NOT_CONVERGED)
    opt = sim._Options()
    lib.sim_default_options(ctypes.byref(opt))
    assert opt.precision == sim.SIM_FP32 and opt.cg_tol == 1e-7 and opt.gravity[2] == -9.81


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2203_11938_amd import sim
    saved = sim._lib
    sim._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            sim.load_library(str(tmp_path / "missing.so"))
    finally:
        sim._lib = saved


def test_adjoint_before_rollout_and_bad_arguments_without_gpu():
    from paper_2203_11938_amd import sim
    lib = sim.load_library()
    # NULL handles and out-of-order calls are rejected before any device work
    assert lib.sim_adjoint(None, None, None, None, None, None, None, None) == sim.SIM_E_INVALID
    assert lib.sim_rollout(None, 1, None, None, None, None, None, None, 0, None,
                           None) == sim.SIM_E_INVALID
    h = ctypes.c_void_p()
    assert lib.sim_create(None, None, None, 0, None, 0.01, None, ctypes.byref(h)) == sim.SIM_E_INVALID
    assert not h.value


def test_matrix_home_option_without_gpu():
    """The solver's matrix home defaults to the library's choice; a value outside
    sim_matrix_home is rejected at option validation, before any device work."""
    import numpy as np
    from paper_2203_11938_amd import sim
    lib = sim.load_library()
    opt = sim._Options()
    lib.sim_default_options(ctypes.byref(opt))
    assert opt.matrix_home == 0 and sim.MATRIX_HOMES[0] == "auto"
    tris = np.array([[0, 1, 2]], np.int32)
    rest = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    mesh = sim._Mesh()
    mesh.n_verts, mesh.n_tris = 3, 1
    mesh.tris = tris.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    mat = sim._Material()
    mat.stretch, mat.bend, mat.density = 1.0, 1.0, 1.0
    for bad in (-1, 4):
        opt.matrix_home = bad
        h = ctypes.c_void_p()
        assert lib.sim_create(ctypes.byref(mesh), rest.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              None, 0, ctypes.byref(mat), 0.01, ctypes.byref(opt),
                              ctypes.byref(h)) == sim.SIM_E_INVALID
        assert not h.value


def _create(lib, sim, tris, rest, pins=None, material=(1.0, 1.0, 1.0), **opts):
    """sim_create through the C ABI with host arrays; returns (status, handle)."""
    import numpy as np
    tris = np.ascontiguousarray(tris, np.int32)
    rest = np.ascontiguousarray(rest, np.float64)
    mesh = sim._Mesh()
    mesh.n_verts, mesh.n_tris = rest.shape[0], tris.shape[0]
    mesh.tris = tris.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    mat = sim._Material()
    mat.stretch, mat.bend, mat.density = material
    opt = sim._Options()
    lib.sim_default_options(ctypes.byref(opt))
    for k, v in opts.items():
        setattr(opt, k, v)
    p = None
    n = 0
    if pins is not None:
        pins = np.ascontiguousarray(pins, np.int32)
        p = pins.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        n = pins.size
    h = ctypes.c_void_p()
    st = lib.sim_create(ctypes.byref(mesh), rest.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        p, n, ctypes.byref(mat), 0.01, ctypes.byref(opt), ctypes.byref(h))
    return st, h


def test_create_time_failures_without_gpu():
    """Mesh and argument errors are found on the host, before any device work: a rest
    triangle of zero area (SIM_E_MESH), a pin index outside the mesh and a negative
    air density (SIM_E_INVALID); no handle is returned."""
    import numpy as np
    from paper_2203_11938_amd import sim, workloads as W
    lib = sim.load_library()
    rest, tris = W.grid_sheet(3)
    flat = rest.copy()
    flat[4] = 0.5 * (flat[3] + flat[5])   # the two triangles on the middle row's left
    flat[[0, 1, 2], 1] = flat[3, 1]        # lie on one line: zero area
    st, h = _create(lib, sim, tris, flat)
    assert st == sim.SIM_E_MESH and not h.value
    st, h = _create(lib, sim, tris, rest, pins=[0, 9])
    assert st == sim.SIM_E_INVALID and not h.value
    st, h = _create(lib, sim, tris, rest, pins=[-1])
    assert st == sim.SIM_E_INVALID and not h.value
    st, h = _create(lib, sim, tris, rest, air_density=-1.0)
    assert st == sim.SIM_E_INVALID and not h.value
    st, h = _create(lib, sim, np.array([[0, 1, 1]]), rest)
    assert st == sim.SIM_E_MESH and not h.value
    # an unknown material model, and the anisotropic model with the tension membrane
    st, h = _create(lib, sim, tris, rest, material_model=2)
    assert st == sim.SIM_E_INVALID and not h.value
    st, h = _create(lib, sim, tris, rest, material_model=sim.SIM_MATERIAL_WANG,
                    membrane_system=sim.SIM_MEMBRANE_TENSION)
    assert st == sim.SIM_E_INVALID and not h.value


def test_material_model_defaults_and_layout():
    """The default model is the isotropic one; the anisotropic material vector is the
    stretch table, the bend table and the density, in that order."""
    import numpy as np
    from paper_2203_11938_amd import sim
    lib = sim.load_library()
    opt = sim._Options()
    lib.sim_default_options(ctypes.byref(opt))
    assert opt.material_model == sim.SIM_MATERIAL_ISOTROPIC
    St = np.arange(24.0).reshape(4, 6)
    Bt = 100.0 + np.arange(15.0).reshape(3, 5)
    v = sim.wang_material(St, Bt, 0.2)
    assert v.shape == (sim.SIM_WANG_PARAMS,)
    assert np.array_equal(v[:24], St.ravel()) and np.array_equal(v[24:39], Bt.ravel())
    assert v[39] == 0.2
