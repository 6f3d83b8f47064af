"""C-ABI boundary on the CPU: exported symbols and host-only logic (no GPU call is made).

bcm_mesh_create and bcm_plan_create run entirely on the host, so mesh validation, option
checks and workspace sizing are exercised here; everything that touches device memory is in
the gpu-marked tests.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1808_04099_amd import _lib as L
    return L, L.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "bcm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = _declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in bcm.h but not exported"
        assert name in L.EXPORTS, f"{name} has no binding in _lib.py"


def _desc(m, **override):
    L, _ = _lib()
    arrs = dict(origin=np.ascontiguousarray(m.origin, np.float64),
                level=np.ascontiguousarray(m.level, np.int8),
                nbr=np.ascontiguousarray(m.nbr, np.int32),
                face_bc=np.ascontiguousarray(m.face_bc, np.int8))
    arrs.update(override)
    d = L.MeshDesc(m.n_cubes if "n_cubes" not in override else override["n_cubes"],
                   override.get("n", m.n),
                   arrs["origin"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   arrs["level"].ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                   override.get("root_edge", m.root_edge),
                   arrs["nbr"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   arrs["face_bc"].ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return d, arrs


def _create(m, **override):
    _, lib = _lib()
    d, keep = _desc(m, **override)
    h = ctypes.c_void_p()
    st = lib.bcm_mesh_create(ctypes.byref(d), ctypes.byref(h))
    msg = lib.bcm_last_error().decode()
    if st == 0:
        lib.bcm_mesh_destroy(h)
    return st, msg


@pytest.mark.parametrize("which", ["channel", "open", "multilevel"])
def test_valid_meshes_are_accepted(which):
    m = {"channel": lambda: uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC),
         "open": lambda: uniform_mesh((2, 2, 2), 0.5, 8, OPEN_BC),
         "multilevel": lambda: configs.multilevel_small()["mesh"]}[which]()
    assert _create(m)[0] == 0


def test_invalid_meshes_are_rejected_with_a_reason():
    m = uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC)
    nbr = m.nbr.copy()
    nbr[0, 1, 0] = 3                       # wrong +x neighbour (not adjacent / not reciprocal)
    st, msg = _create(m, nbr=nbr)
    assert st == -2 and "cube 0 face 1" in msg
    nbr = m.nbr.copy()
    nbr[0, 1, 1] = 2                       # two slots filled: neither 1 nor 4 neighbours
    assert _create(m, nbr=nbr)[0] == -2
    bc = m.face_bc.copy()
    bc[m.nbr[:, :, 0] < 0] = 3             # every boundary face slip: singular Poisson problem
    st, msg = _create(m, face_bc=bc)
    assert st == -2 and "OUTFLOW" in msg
    bc = m.face_bc.copy()
    bc[0, 0] = 0                           # boundary face without a kind
    assert _create(m, face_bc=bc)[0] == -2
    lv = m.level.copy()
    lv[5] = 2                              # level jump
    assert _create(m, level=lv)[0] == -2
    assert _create(m, n=6)[0] == -1        # unsupported cells per edge
    assert _create(m, root_edge=-1.0)[0] == -1


def test_multilevel_slot_order_is_checked():
    m = configs.multilevel_small()["mesh"]
    nbr = m.nbr.copy()
    c, f = np.argwhere(nbr[:, :, 1] >= 0)[0]
    nbr[c, f, [0, 1]] = nbr[c, f, [1, 0]]  # swap two sub-neighbours
    st, msg = _create(m, nbr=nbr)
    assert st == -2, msg


def test_plan_workspace_and_options():
    L, lib = _lib()
    m = uniform_mesh((4, 2, 2), 0.25, 16, CHANNEL_BC)
    d, keep = _desc(m)
    mh = ctypes.c_void_p()
    assert lib.bcm_mesh_create(ctypes.byref(d), ctypes.byref(mh)) == 0
    try:
        sizes = {}
        for prec in (0, 1, 2):
            o = L.SolverOpts()
            lib.bcm_default_opts(ctypes.byref(o))
            o.precision = prec
            ph = ctypes.c_void_p()
            nb = ctypes.c_size_t()
            assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == 0
            sizes[prec] = nb.value
            # unbound plan: every solver entry point refuses with BCM_ERR_WORKSPACE
            assert lib.bcm_apply_laplacian(ph, None, None, None) == -3
            lib.bcm_plan_destroy(ph)
        cells = m.n_cells
        # FP64 needs at least: 3 u* + b + lambda + 4 Krylov vectors of 8 bytes per cell
        assert sizes[0] >= cells * 8 * 9
        # mixed keeps FP32 Krylov vectors, FP32 fields shrink u*: workspaces shrink
        assert sizes[2] < sizes[1] < sizes[0]
        o = L.SolverOpts()
        lib.bcm_default_opts(ctypes.byref(o))
        assert (o.max_iter, o.max_outer, o.coarse_solver, o.coarse_cycles, o.graph_split,
                o.prolong, o.check_every) == (50, 10, 1, 1, -1, 1, 1)
        o.graph_split = -2
        ph = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == -1
        lib.bcm_default_opts(ctypes.byref(o))
        o.prolong = 2
        assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == -1
        lib.bcm_default_opts(ctypes.byref(o))
        o.krylov = 3
        assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == -1
        lib.bcm_default_opts(ctypes.byref(o))
        o.check_every = 0
        assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == -1
        lib.bcm_default_opts(ctypes.byref(o))
        o.tol = -1.0
        ph = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        assert lib.bcm_plan_create(mh, ctypes.byref(o), ctypes.byref(ph), ctypes.byref(nb)) == -1
        assert "invalid solver options" in lib.bcm_last_error().decode()
    finally:
        lib.bcm_mesh_destroy(mh)


def test_status_strings_and_timer_names():
    _, lib = _lib()
    assert lib.bcm_status_string(0) == b"BCM_OK"
    assert lib.bcm_status_string(-4) == b"BCM_ERR_NONFINITE"
    from paper_1808_04099_amd import timing_names
    names = timing_names()
    assert "postsmooth16" in names and "coarse" in names


@pytest.mark.parametrize("which", ["uniform", "multilevel"])
def test_boundary_face_with_a_cube_across_is_rejected(which):
    """A face whose neighbour slots are empty must lie on the domain boundary: unlinking two
    touching cubes and marking both faces as open boundaries is caught by the geometry check."""
    m = (uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC) if which == "uniform"
         else configs.multilevel_small()["mesh"])
    nbr, bc = m.nbr.copy(), m.face_bc.copy()
    if which == "uniform":
        c, f = 0, 1
    else:                                  # a coarse face with four finer neighbours
        c, f = map(int, np.argwhere(nbr[:, :, 1] >= 0)[0])
    others = [int(o) for o in nbr[c, f] if o >= 0]
    nbr[c, f] = -1
    bc[c, f] = 1
    for o in others:
        nbr[o, f ^ 1] = -1
        bc[o, f ^ 1] = 1
    st, msg = _create(m, nbr=nbr, face_bc=bc)
    assert st == -2 and "a cube lies across it" in msg, msg


def test_overlapping_cubes_are_rejected():
    m = uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC)
    origin = m.origin.copy()
    origin[1] = origin[0] + 0.1            # off the level lattice
    st, msg = _create(m, origin=origin)
    assert st == -2, msg
