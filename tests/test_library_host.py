"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/hdg.h declares, and
reject invalid arguments and invalid meshes before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import Mesh, TET

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "hdg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = hdg.load_library()
    declared = _header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(hdg.EXPORTS) == declared


def _create(mesh, N=2, bc=1, precision=0, hanging=None):
    lib = hdg.load_library()
    xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
    et = np.ascontiguousarray(mesh.etype, dtype=np.int8)
    ev = np.ascontiguousarray(mesh.everts, dtype=np.int64)
    ka = np.ascontiguousarray(mesh.kappa, dtype=np.float64)
    rh = np.ascontiguousarray(mesh.rho, dtype=np.float64)
    hg = np.ascontiguousarray(np.zeros((0, 3)) if hanging is None else hanging, dtype=np.int64).reshape(-1, 3)
    bf = getattr(mesh, "bc_face", None)
    bf = None if bf is None else np.ascontiguousarray(bf, dtype=np.int8)
    m = hdg.HdgMesh(xyz.shape[0], xyz.ctypes.data, et.shape[0], et.ctypes.data, ev.ctypes.data,
                    ka.ctypes.data, rh.ctypes.data, bc, None if bf is None else bf.ctypes.data,
                    hg.shape[0], hg.ctypes.data if hg.shape[0] else None)
    h = ctypes.c_void_p()
    rc = lib.hdg_create(ctypes.byref(h), ctypes.byref(m), N, precision, None)
    return rc, h, lib.hdg_last_error(None).decode()


def _tets(verts, xyz):
    n = len(verts)
    ev = -np.ones((n, 8), dtype=np.int64)
    for i, v in enumerate(verts):
        ev[i, :4] = v
    return Mesh(xyz=np.asarray(xyz, dtype=np.float64), etype=np.full(n, TET, dtype=np.int8), everts=ev,
                kappa=np.ones(n), rho=np.ones(n))


XYZ = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]]


@pytest.mark.parametrize("N", [0, 6, 9])
def test_create_rejects_unsupported_order(N):
    rc, h, msg = _create(_tets([[0, 1, 2, 3]], XYZ), N=N)
    assert rc == -1 and not h.value and "order" in msg


@pytest.mark.parametrize("precision", [-1, 5, 7])
def test_create_rejects_unknown_precision(precision):
    rc, h, msg = _create(_tets([[0, 1, 2, 3]], XYZ), precision=precision)
    assert rc == -1 and not h.value and "precision" in msg


def test_create_rejects_non_manifold_face():
    # three tetrahedra sharing the face (0,1,2)
    rc, h, msg = _create(_tets([[0, 1, 2, 3], [0, 2, 1, 4], [0, 1, 2, 5]], XYZ))
    assert rc == -2 and not h.value and "more than two" in msg


def test_create_rejects_bad_vertex_id():
    rc, h, msg = _create(_tets([[0, 1, 2, 17]], XYZ))
    assert rc == -1 and "vertex" in msg


def test_create_rejects_bad_material_and_bc():
    m = _tets([[0, 1, 2, 3]], XYZ)
    m.rho[:] = 0.0
    rc, _, msg = _create(m)
    assert rc == -1 and "rho" in msg
    rc, _, msg = _create(_tets([[0, 1, 2, 3]], XYZ), bc=7)
    assert rc == -1 and "boundary" in msg


def test_create_rejects_bad_face_boundary_condition():
    m = _tets([[0, 1, 2, 3]], XYZ)
    m.bc_face = np.full((1, 6), -1, dtype=np.int8)
    m.bc_face[0, 2] = 3
    rc, h, msg = _create(m)
    assert rc == hdg.EINVAL and not h.value and "boundary condition" in msg


def test_binding_fails_loudly_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(hdg.HdgError):
        hdg.Solver(_tets([[0, 1, 2, 3]], XYZ), 2)


def test_calls_on_a_null_context_are_rejected():
    lib = hdg.load_library()
    t = ctypes.c_double()
    n = ctypes.c_int64()
    buf = (ctypes.c_uint8 * 64)()
    assert lib.hdg_get_time(None, ctypes.byref(t)) == hdg.EINVAL
    assert lib.hdg_set_time(None, 1.0) == hdg.EINVAL
    assert lib.hdg_check_finite(None) == hdg.EINVAL
    assert lib.hdg_advance(None, 1.0, hdg.STEPPER_LSERK4, 0.5, 0, ctypes.byref(n)) == hdg.EINVAL
    assert lib.hdg_checkpoint_size(None, ctypes.byref(n)) == hdg.EINVAL
    assert lib.hdg_checkpoint_save(None, buf, 64) == hdg.EINVAL
    assert lib.hdg_checkpoint_load(None, buf, 64) == hdg.EINVAL
    assert lib.hdg_project_noalloc(None, 0, None, None, None, None) == hdg.EINVAL
    assert lib.hdg_project(None, 0, None, None, None, None) == hdg.EINVAL
    assert lib.hdg_mrab_level_info(None, buf) == hdg.EINVAL
    assert lib.hdg_trace_constants(None, buf) == hdg.EINVAL
    assert lib.hdg_set_dt_mode(None, hdg.DT_ELEMENT) == hdg.EINVAL
    assert lib.hdg_autotune(None, 5, None) == hdg.EINVAL


def test_header_scratch_size_matches_binding():
    src = open(os.path.join(ROOT, "include", "hdg.h")).read()
    m = re.search(r"#define HDG_PROJECT_SCRATCH_BYTES \((\d+) \* (\d+) \* (\d+)\)", src)
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == hdg.PROJECT_SCRATCH_BYTES


# A coarse tetrahedron below the triangle (0, 1, 2) of z = 0 and four fine
# tetrahedra above the four triangles of its midpoint subdivision (hanging
# vertices 3, 4, 5 at the edge midpoints, apex 6).
NC_XYZ = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.5, 0, 0], [0.5, 0.5, 0], [0, 0.5, 0], [0.2, 0.2, 0.5],
          [0.2, 0.2, -1]]
NC_TETS = [[0, 1, 2, 7], [0, 3, 5, 6], [1, 4, 3, 6], [2, 5, 4, 6], [3, 4, 5, 6]]
NC_HANG = [[3, 0, 1], [4, 1, 2], [5, 2, 0]]


def test_create_rejects_hanging_vertex_off_its_midpoint():
    xyz = np.array(NC_XYZ, dtype=np.float64)
    xyz[4, 0] += 1e-6
    rc, h, msg = _create(_tets(NC_TETS, xyz), hanging=NC_HANG)
    assert rc == hdg.EMESH and not h.value and "midpoint" in msg


def test_create_rejects_bad_hanging_rows():
    rc, _, msg = _create(_tets(NC_TETS, NC_XYZ), hanging=[[3, 0, 0]])
    assert rc == hdg.EINVAL and "hanging" in msg
    rc, _, msg = _create(_tets(NC_TETS, NC_XYZ), hanging=[[3, 0, 99]])
    assert rc == hdg.EINVAL and "hanging" in msg


def test_create_rejects_a_refined_face_with_a_missing_sub_face():
    # the middle sub-face (3, 4, 5) has no element
    rc, _, msg = _create(_tets(NC_TETS[:4], NC_XYZ), hanging=NC_HANG)
    assert rc == hdg.EMESH and "sub-face" in msg


def test_create_accepts_the_refined_face_up_to_the_device():
    # the non-conforming set-up is host work; without a GPU the call stops at
    # the first device query, with a HIP error rather than a mesh error
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, _, msg = _create(_tets(NC_TETS, NC_XYZ), hanging=NC_HANG)
    assert rc == hdg.EHIP, msg
