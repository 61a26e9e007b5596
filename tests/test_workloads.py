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
