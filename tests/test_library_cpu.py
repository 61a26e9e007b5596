"""Host-side checks of the HIP library (no GPU needed): it loads, exports every
symbol declared in include/vof.h, its geometry code (compiled for the host as
well) agrees with the oracle, and its error paths report cleanly."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1305_3417_amd as vof
from tests import exact_geometry as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TET_F = [[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]]


def _header_functions():
    src = open(os.path.join(ROOT, "include", "vof.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vof_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol():
    L = vof.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vof.EXPORTED)
    assert "gfx950" in vof.vof_version()


def test_selftest_clip_matches_oracle(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(1500):
        T = rng.random((4, 3))
        k = int(rng.integers(0, 8))
        planes = np.concatenate([rng.normal(size=(k, 3)), rng.uniform(0, 0.8, (k, 1))], 1)
        a = vof.vof_selftest_tet_clip(T, planes)
        Tt = T.copy()
        if np.linalg.det(Tt[1:] - Tt[0]) < 0:
            Tt[[2, 3]] = Tt[[3, 2]]
        b = (oracle_mod.clip_volume(Tt, TET_F, planes) if k
             else abs(np.linalg.det(T[1:] - T[0])) / 6)
        assert abs(a - b) <= 1e-15


def test_selftest_clip_degenerate_dyadic_exact():
    """Coplanar faces, vertices on planes: exact rational reference."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        T = rng.integers(0, 9, (4, 3)) / 8.0
        if abs(np.linalg.det(T[1:] - T[0])) < 1e-9:
            continue
        k = int(rng.integers(1, 7))
        planes = np.concatenate([rng.integers(-2, 3, (k, 3)), rng.integers(0, 9, (k, 1)) / 8.0], 1)
        planes = planes[np.abs(planes[:, :3]).sum(1) > 0]
        a = vof.vof_selftest_tet_clip(T, planes)
        exact = float(X.tet_halfspaces_volume(T, planes))
        assert abs(a - exact) <= 1e-15


def test_selftest_closed_forms_match_oracle(oracle_mod):
    """The register path (up to four planes, the tet's kept part split into
    tetrahedra and carried as vertex distances) against the oracle's
    clip-and-cap, on random tets and planes."""
    rng = np.random.default_rng(21)
    for _ in range(4000):
        T = rng.random((4, 3))
        k = int(rng.integers(0, 5))
        planes = np.concatenate([rng.normal(size=(k, 3)), rng.uniform(0, 0.8, (k, 1))], 1)
        a = vof.vof_selftest_tet_clip_closed(T, planes)
        Tt = T.copy()
        if np.linalg.det(Tt[1:] - Tt[0]) < 0:
            Tt[[2, 3]] = Tt[[3, 2]]
        b = (oracle_mod.clip_volume(Tt, TET_F, planes) if k
             else abs(np.linalg.det(T[1:] - T[0])) / 6)
        assert abs(a - b) <= 1e-15, (k, a, b)


def test_selftest_closed_forms_degenerate_dyadic_exact():
    """Vertices on planes, coplanar faces and parallel planes, against exact
    rational volumes; every count of kept vertices occurs at every level."""
    rng = np.random.default_rng(22)
    seen = 0
    for _ in range(1500):
        T = rng.integers(0, 9, (4, 3)) / 8.0
        if abs(np.linalg.det(T[1:] - T[0])) < 1e-9:
            continue
        k = int(rng.integers(1, 5))
        planes = np.concatenate([rng.integers(-2, 3, (k, 3)), rng.integers(0, 9, (k, 1)) / 8.0], 1)
        planes = planes[np.abs(planes[:, :3]).sum(1) > 0]
        a = vof.vof_selftest_tet_clip_closed(T, planes)
        exact = float(X.tet_halfspaces_volume(T, planes))
        assert abs(a - exact) <= 1e-15, (T, planes, a, exact)
        seen += exact > 0
    assert seen > 300


def test_selftest_closed_forms_refuse_five_planes():
    T = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    planes = np.array([[1, 0, 0, 0.5], [0, 1, 0, 0.5], [0, 0, 1, 0.5], [1, 1, 1, 0.9],
                       [-1, 0, 0, 0.0]])
    assert np.isnan(vof.vof_selftest_tet_clip_closed(T, planes))
    # four planes: the cube [0, 1/2]^3 below x + y + z = 0.9 (a corner tet of
    # legs 0.9 minus three corner tets of legs 0.4 beyond the cube faces)
    v4 = 0.9 ** 3 / 6 - 3 * 0.4 ** 3 / 6
    assert abs(vof.vof_selftest_tet_clip_closed(T, planes[:4]) - v4) < 1e-16
    # the cube [0, 1/2]^3 minus its corner beyond x + y + z = 1
    assert abs(vof.vof_selftest_tet_clip_closed(T, planes[:3]) - 5 / 48) < 1e-17


def test_selftest_clip_near_degenerate_sequences():
    """Planes through vertices, edges and earlier cut points of the tet, each
    offset moved by rounding-sized amounts (1e-17 relative) and applied in
    sequences of six: coincident vertices and sign noise on them must give a
    consistent polytope (no NaN) whose volume is the exact one to 1e-14."""
    rng = np.random.default_rng(23)
    for _ in range(400):
        T = rng.integers(0, 9, (4, 3)) / 8.0
        if abs(np.linalg.det(T[1:] - T[0])) < 1e-9:
            continue
        planes, exact_planes = [], []
        for _ in range(6):
            nrm = rng.integers(-3, 4, 3).astype(float)
            if not nrm.any():
                nrm[0] = 1.0
            # through a vertex, or through the midpoint of an edge
            if rng.random() < 0.5:
                x = T[rng.integers(4)]
            else:
                i, j = rng.choice(4, 2, replace=False)
                x = 0.5 * (T[i] + T[j])
            s0 = float(nrm @ x)
            exact_planes.append(list(nrm) + [s0])
            noise = rng.choice([-1.0, 0.0, 1.0]) * 1e-17 * (abs(s0) + 1.0)
            planes.append(list(nrm) + [s0 + noise])
        a = vof.vof_selftest_tet_clip(T, np.array(planes))
        exact = float(X.tet_halfspaces_volume(T, exact_planes))
        assert np.isfinite(a), (T, planes)
        assert abs(a - exact) <= 1e-14, (T, planes, a, exact)


def test_selftest_clip_box_capacity():
    """A tet cut by the six planes of a box and an oblique plane stays within
    the polytope capacity."""
    T = np.array([[-0.2, -0.1, -0.3], [1.3, 0.1, 0.2], [0.2, 1.2, -0.1], [0.4, 0.3, 1.4]])
    planes = X.box_planes((0, 0, 0), (1, 1, 1)) + [(1, 1, 1, 1.5)]
    a = vof.vof_selftest_tet_clip(T, np.array(planes, float))
    assert np.isfinite(a)
    assert abs(a - float(X.tet_halfspaces_volume(T, planes))) < 1e-15


def test_no_device_error_is_clean():
    """Without a visible GPU the context call fails with VOF_EDEVICE and a
    message, and never aborts.  (Skipped where a GPU is present.)"""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(vof.VofError) as e:
        vof.vof_context_create(0)
    assert e.value.code == vof.VOF_EDEVICE
    assert "device" in vof.vof_last_error()


def test_null_arguments_rejected():
    L = vof.lib()
    assert L.vof_mesh_upload(None, None, None) == vof.VOF_EINVAL
    assert L.vof_set_alpha(None, None, 0) == vof.VOF_EINVAL
    assert L.vof_advect(None, 1, None, None) == vof.VOF_EINVAL
    assert np.isnan(L.vof_selftest_tet_clip(None, 0, None))
    assert np.isnan(L.vof_selftest_tet_clip_closed(None, 0, None))
    assert vof.vof_profile_kernel_name(0) == "reset"
    assert vof.vof_profile_kernel_name(99) is None
