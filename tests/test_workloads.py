"""The synthetic inputs: face fluxes discretely divergence free (eq. 2.4),
equal to the velocity's flux through each face, and the adaptive Courant
schedule of the shear test (Section 4.2.2) as its rule states."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from workloads import fields


def _cell_divergence(m, F):
    div = np.zeros(m.n_cells)
    np.add.at(div, m.owner, F)
    np.add.at(div, m.neighbour, -F[:m.n_internal])
    return div


@pytest.mark.parametrize("make", [lambda: W.deform3d(8, steps=1), lambda: W.rotate_tets(4, steps=1),
                                  lambda: W.shear3d(8, steps=1), lambda: W.disc2d(8, steps=1)])
def test_fluxes_divergence_free(make):
    w = make()
    div = _cell_divergence(w.mesh, w.F0)
    assert np.abs(div).max() <= 1e-15 * max(np.abs(w.F0).max(), 1e-300)


def _face_quadrature_flux(m, vel, order=8):
    """∫ U·n dA over each planar quad face by tensor Gauss-Legendre (bilinear map)."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    t = 0.5 * (xg + 1.0)
    wq = 0.5 * wg
    out = np.zeros(m.n_faces)
    for f in range(m.n_faces):
        P = m.points[m.face_points[m.face_offsets[f]:m.face_offsets[f + 1]]]
        acc = 0.0
        for i, u in enumerate(t):
            for j, v in enumerate(t):
                x = (1 - u) * (1 - v) * P[0] + u * (1 - v) * P[1] + u * v * P[2] + (1 - u) * v * P[3]
                xu = (1 - v) * (P[1] - P[0]) + v * (P[2] - P[3])
                xv = (1 - u) * (P[3] - P[0]) + u * (P[2] - P[1])
                acc += wq[i] * wq[j] * vel(x[None])[0] @ np.cross(xu, xv)
        out[f] = acc
    return out


def test_shear_fluxes_are_velocity_fluxes():
    """F_f from the vector potential equals ∫ U0·n over the face (24x24 Gauss;
    the cone of the axial component has its kink on face corners, where both
    quadratures converge algebraically, hence 1e-8 of the face area)."""
    w = W.shear3d(4, steps=1)
    q = _face_quadrature_flux(w.mesh, fields.shear_velocity, order=24)
    S = (1.0 / 4) ** 2
    assert np.abs(w.F0 - q).max() <= 1e-8 * S


def test_shear_velocity_at_known_points():
    x = np.array([[0.5, 0.5, 0.3], [0.25, 0.5, 0.0], [0.5, 0.25, 0.9], [0.0, 0.0, 0.5]])
    U = fields.shear_velocity(x)
    assert np.allclose(U[0], [0.0, 0.0, 1.0], atol=1e-15)          # on the axis: w = u_max
    assert np.allclose(U[1], [0.0, -1.0, 0.25], atol=1e-15)       # r = 1/4: w = (1 - 1/2)^2
    assert np.allclose(U[2], [1.0, 0.0, 0.25], atol=1e-15)
    assert np.allclose(U[3], [0.0, 0.0, (1 - np.sqrt(0.5) / 0.5) ** 2], atol=1e-15)


def test_courant_schedule_rule():
    """dt_0 = Co h / Umax; dt_{n+1} = min(Co h / (Umax |s_n|), 2 dt_0) with
    s_n = cos(pi (t_n + dt_n/2) / T); the run ends at T; the Courant number of
    every step stays at Co, within the one-step lag."""
    Umax, h, T, co = 1.3, 1.0 / 32, 3.0, 0.5
    dt, sc = W.courant_schedule(Umax, h, T, co)
    t = np.concatenate([[0.0], np.cumsum(dt)])
    assert abs(t[-1] - T) <= 1e-12
    assert dt[0] == co * h / Umax
    assert np.allclose(sc, np.cos(np.pi * (t[:-1] + 0.5 * dt) / T), rtol=0, atol=1e-15)
    for n in range(len(dt) - 2):
        assert dt[n + 1] == min(co * h / (Umax * abs(sc[n])), 2.0 * dt[0])
    courant = dt * Umax * np.abs(sc) / h
    assert courant.max() <= co * 1.05
    # the slowed-down middle of the run uses the longer steps
    assert dt.max() == 2.0 * dt[0] and len(dt) < T / dt[0]


def test_tet_step_keeps_cell_courant_at_half(oracle_mod):
    """The jittered-tet rotation's step: every cell's Courant number
    (1/2) sum_f |F_f| dt / V_c, with V_c from the oracle's own geometry, is at
    most 0.5, and the largest is within one step of it (dt = 1 / N)."""
    w = W.rotate_tets(12, steps=2, sample=2)
    V = oracle_mod.Oracle(w.mesh).geometry()[0]
    m = w.mesh
    S = np.zeros(m.n_cells)
    np.add.at(S, m.owner, np.abs(w.F0))
    np.add.at(S, m.neighbour, np.abs(w.F0[:m.n_internal]))
    co = 0.5 * S * w.dt[0] / V
    N = w.meta["steps_per_rev"]
    assert w.dt[0] == 1.0 / N
    assert co.max() <= 0.5 * (1 + 1e-12)
    assert co.max() >= 0.5 * (N - 1) / N
    # the velocity-over-spacing step this replaces would give cells above 1
    assert (0.5 * S / V).max() / (9 * 12) > 1.0


# --------------------------------------------------------------------------
# 2:1 refined hexahedral meshes
# --------------------------------------------------------------------------

def _sphere_band_mask(n, centre=(0.45, 0.5, 0.55), r=0.3, width=0.6):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    xc = (np.stack([i.ravel(), j.ravel(), k.ravel()], 1) + 0.5) / n
    d = np.abs(np.linalg.norm(xc - np.asarray(centre), axis=1) - r)
    return d < width / n


def test_refined_mesh_is_conforming():
    """Every cell's outward faces close up: each directed edge of its surface
    has its reverse in the same cell (so faces list the points neighbours add
    on shared edges), the area vectors sum to zero, volumes and centroids are
    those of the generating boxes, and no cell has more than 15 faces or a
    face more than 8 points."""
    from workloads.refine import refine_hex
    n = 6
    m, parent, (coff, cells) = refine_hex(n, _sphere_band_mask(n))
    assert m.meta["refined"] > 0
    off = m.face_offsets
    faces_of = [[] for _ in range(m.n_cells)]
    for f in range(m.n_faces):
        ps = m.face_points[off[f]:off[f + 1]].tolist()
        faces_of[m.owner[f]].append(ps)
        if f < m.n_internal:
            faces_of[m.neighbour[f]].append(ps[::-1])
    for c, fs in enumerate(faces_of):
        assert len(fs) <= 15
        edges = {}
        for ps in fs:
            assert 4 <= len(ps) <= 8
            for a, b in zip(ps, ps[1:] + ps[:1]):
                edges[(a, b)] = edges.get((a, b), 0) + 1
        assert all(v == 1 and edges.get((b, a)) == 1 for (a, b), v in edges.items()), c
        # area vectors of the outward faces sum to zero; volume by divergence
        X = m.points
        Ssum = np.zeros(3)
        vol = 0.0
        for ps in fs:
            P = X[ps]
            cf = P.mean(axis=0)
            for a, b in zip(P, np.roll(P, -1, axis=0)):
                Ssum += 0.5 * np.cross(a - cf, b - cf)
                vol += np.dot(cf, np.cross(a - cf, b - cf)) / 6.0
        assert np.abs(Ssum).max() < 1e-15
        assert abs(vol - np.prod(m.cell_hi[c] - m.cell_lo[c])) < 1e-15
    # parent and children maps agree
    assert coff[-1] == m.n_cells and np.array_equal(np.repeat(np.arange(n ** 3), np.diff(coff)), parent)
    for o in range(n ** 3):
        kids = cells[coff[o]:coff[o + 1]]
        lo = m.cell_lo[kids].min(axis=0)
        hi = m.cell_hi[kids].max(axis=0)
        i, j, k = o % n, (o // n) % n, o // (n * n)
        assert np.allclose(lo, np.array([i, j, k]) / n) and np.allclose(hi, np.array([i + 1, j + 1, k + 1]) / n)


def test_refinement_closure():
    """No coarse cell is left with more than three refined face neighbours."""
    from workloads.refine import close_refinement
    n = 7
    rng = np.random.default_rng(3)
    m = close_refinement(n, rng.random(n ** 3) < 0.3).reshape(n, n, n)
    cnt = np.zeros(m.shape, dtype=int)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax], hi[ax] = slice(0, n - 1), slice(1, n)
        cnt[tuple(lo)] += m[tuple(hi)]
        cnt[tuple(hi)] += m[tuple(lo)]
    assert cnt[~m].max(initial=0) <= 3
