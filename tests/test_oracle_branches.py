"""Pins of the oracle's correction-clamp and vanishing-gradient branches.

Both branches are readings (the paper treats neither): a face whose
correction target lies beyond the extremum of its swept volume on the
monotone branch is clamped there and carries its polyhedron's phase fraction
of F dt when that polyhedron holds at least a quarter of F dt, else the
upwind (donor) cell's fraction (Section 2.3 assumes the correction always
converges); an
interface cell whose gradient vanishes is treated as homogeneous,
contributing alpha_c |T ∩ C_c| (Algorithm 1 has no normal to offer).  The
pins use inputs for which the mathematics fixes the answer independently of
either implementation:

* alpha uniform: every cell is an interface cell with zero gradient, so every
  flux polyhedron inside the domain carries alpha times its volume F dt, and
  a clamped face alpha F dt as well (its phase fraction alpha scaled to
  F dt).  An empty/full reading of the homogeneous cell, or a clamped face
  with a missing or inverted scale, fails it.
* fluxes k times U.S under a translation: the swept volume is linear in
  lambda, so lambda = k up to the branch end (32 plain sweeps) and a clamp
  to the plain sweep (lambda = 1) beyond it; with k = 40 every face is
  clamped and the whole update is the donor-cell (first-order upwind)
  update, written out here with numpy.
* one symmetric cell in an empty box under translation: the cell is
  homogeneous by symmetry, the outflow prism lies in it, so it keeps
  alpha (1 - u dt / h) and its downstream neighbour gets alpha u dt / h.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.common import vphase_tolerance


def _interior_faces(w):
    """Faces with flux none of whose points lies on the box: their flux
    polyhedra (Co 0.5) stay inside the domain."""
    m = w.mesh
    onb = W.boundary_points(m)
    n = np.diff(m.face_offsets)
    face_of = np.repeat(np.arange(m.n_faces), n)
    touch = np.zeros(m.n_faces, bool)
    np.logical_or.at(touch, face_of, onb[m.face_points])
    return np.flatnonzero(~touch & (w.F0 != 0))


def test_uniform_alpha_faces_carry_alpha_times_flux(oracle_mod):
    """Deformation field (eq. 4.6) on 16^3, alpha = 0.37: every cell is of the
    vanishing-gradient class, clamped faces occur, and every interior face,
    clamped or not, carries 0.37 F dt; interior cells keep 0.37 (eq. 2.4)."""
    w = W.uniform_alpha(W.deform3d(16, steps=1), 0.37)
    o = oracle_mod.Oracle(w.mesh)
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    assert (r["rec"]["cls"] == 3).all()
    sdt = w.dt[0] * w.scale[0]
    T = w.F0 * sdt
    tol = vphase_tolerance(w, V, sdt, S, Up)
    faces = _interior_faces(w)
    clamped = faces[r["status"][faces] == 1]
    print(f"[uniform] {faces.size} interior faces, {clamped.size} clamped", flush=True)
    assert clamped.size > 20
    # clamped polyhedra here hold half of F dt or more: scaled, not donor faces
    assert (r["kind"][faces] == 3).all()
    err = np.abs(r["vphase"][faces] - 0.37 * T[faces])
    assert (err <= tol[faces]).all(), (err / tol[faces]).max()
    # a clamped face's own swept volume is not F dt: only the scaling gives it F dt
    vlam = np.array([o.flux_volume(f, w.dt[0], w.scale[0], r["lam"][f]) for f in clamped])
    assert (np.abs(vlam - T[clamped]) > 1e3 * tol[clamped]).any()
    # cells whose faces are all interior keep alpha to the faces' bounds
    m = w.mesh
    inner = np.zeros(m.n_faces, bool)
    inner[faces] = True
    inner |= w.F0 == 0
    ok = np.ones(m.n_cells, bool)
    np.logical_and.at(ok, m.owner, inner)
    np.logical_and.at(ok, m.neighbour, inner[:m.n_internal])
    bound = np.zeros(m.n_cells)
    np.add.at(bound, m.owner, tol)
    np.add.at(bound, m.neighbour, tol[:m.n_internal])
    cells = np.flatnonzero(ok)
    assert cells.size > 100
    assert (np.abs(r["alpha"][cells] - 0.37) <= bound[cells] / V[cells] + 1e-15).all()


def test_isolated_symmetric_cell_is_homogeneous(oracle_mod):
    """One cell of 0.5 in an empty 8^3 box, translated along +x at Co 0.5:
    its NAG gradient vanishes by symmetry (class 3); after one step it holds
    0.5 (1 - u dt / h) and its downstream neighbour 0.5 u dt / h."""
    w = W.isolated_cell(8, 0.25, 0.5)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    c = w.meta["cell"]
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    cls = r["rec"]["cls"]
    assert cls[c] == 3
    assert (np.delete(cls, c) == 0).all()
    h = 1.0 / 8
    frac = 0.25 * w.dt[0] / h
    expect = np.zeros(w.mesh.n_cells)
    expect[c] = 0.5 * (1 - frac)
    expect[c + 1] = 0.5 * frac
    assert np.abs(r["alpha"] - expect).max() < 1e-15
    # the outflow face carries 0.5 u dt h^2
    m = w.mesh
    f = np.flatnonzero((m.owner[:m.n_internal] == c) & (m.neighbour == c + 1))[0]
    assert r["vphase"][f] == pytest.approx(0.5 * 0.25 * w.dt[0] * h * h, rel=1e-14)
    assert r["status"][f] == 0


@pytest.mark.parametrize("k,status,lam", [(20.0, 0, 20.0), (31.0, 0, 31.0), (33.0, 1, 1.0),
                                          (40.0, 1, 1.0)])
def test_correction_branch_end_at_32_sweeps(oracle_mod, k, status, lam):
    """Translation with F = k U.S_f: V(lambda) = lambda dt U.S_f has no
    extremum, so the branch ends at 32 plain sweeps; a target inside it is
    met at lambda = k, one beyond it clamps to the plain sweep (status 1),
    and with alpha uniform every interior face still carries 0.37 F dt."""
    w = W.scaled_translation(8, k)
    o = oracle_mod.Oracle(w.mesh)
    V, _, S, _ = o.geometry()
    o.set_velocity(w.U0c, w.F0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    faces = _interior_faces(w)
    assert faces.size > 0
    assert (r["status"][faces] == status).all()
    assert np.abs(r["lam"][faces] - lam).max() <= 1e-12 * lam
    T = w.F0 * w.dt[0]
    assert np.abs(r["vphase"][faces] - 0.37 * T[faces]).max() <= 1e-13 * np.abs(T[faces]).max()


def donor_update(w, alpha):
    """The first-order upwind (donor-cell) step written out: every face with
    flux carries the alpha of the cell its flux leaves times F dt (nothing
    for inflow through a boundary face); alpha -= (1/V) sum of the signed
    face volumes (owner +, neighbour -)."""
    m = w.mesh
    T = w.F0 * w.dt[0] * w.scale[0]
    ni = m.n_internal
    donor = np.where(T > 0, m.owner, np.concatenate([m.neighbour, np.full(m.n_faces - ni, -1)]))
    vph = np.where(donor >= 0, alpha[np.maximum(donor, 0)] * T, 0.0)
    V = np.prod(m.cell_hi - m.cell_lo, axis=1)
    acc = np.zeros(m.n_cells)
    np.add.at(acc, m.owner, vph)
    np.add.at(acc, m.neighbour, -vph[:ni])
    return alpha - acc / V, vph


def test_unreachable_targets_take_the_donor_cell(oracle_mod):
    """Fluxes 40 U.S_f (beyond the branch end) on a random alpha field: every
    face with flux is clamped, and the step is the donor-cell update."""
    w = W.scaled_translation(8, 40.0)
    rng = np.random.default_rng(5)
    a0 = rng.uniform(0.05, 0.95, w.mesh.n_cells)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    r = o.step(a0, w.dt[0], w.scale[0])
    flux = w.F0 != 0
    assert (r["status"][flux] == 1).all() and (r["kind"][flux] == 4).all()
    a_ref, v_ref = donor_update(w, a0)
    assert np.array_equal(r["vphase"], v_ref)
    assert np.abs(r["alpha"] - a_ref).max() <= 1e-15


def test_zero_sweep_with_flux_takes_the_donor_cell(oracle_mod):
    """Point velocities all zero but face fluxes non-zero: the swept volume
    vanishes identically (no correction can reach F dt), every face with
    flux is clamped at lambda = 0 and carries its donor cell's alpha F dt."""
    w = W.scaled_translation(8, 1.0)
    w.U0c[:] = 0.0
    rng = np.random.default_rng(6)
    a0 = rng.uniform(0.05, 0.95, w.mesh.n_cells)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    r = o.step(a0, w.dt[0], w.scale[0])
    flux = w.F0 != 0
    assert (r["status"][flux] == 1).all() and (r["lam"][flux] == 0).all()
    a_ref, v_ref = donor_update(w, a0)
    assert np.array_equal(r["vphase"], v_ref)
    assert np.abs(r["alpha"] - a_ref).max() <= 1e-15
