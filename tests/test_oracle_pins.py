"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test states the closed form, invariant or independent exact computation
it uses.  None of them re-types the oracle's own formula.
"""
from __future__ import annotations

from fractions import Fraction as Q

import numpy as np
import pytest

import workloads as W
from tests import exact_geometry as X

CUBE_V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                   [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
CUBE_F = [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [2, 3, 7, 6], [1, 2, 6, 5], [0, 4, 7, 3]]
TET_F = [[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]]


# --------------------------------------------------------------------------
# plane clipping and capping (Section 2.1)
# --------------------------------------------------------------------------

def test_clip_truncated_cube_closed_form(oracle_mod):
    """|cube ∩ {m.x <= s}| = sum_v (-1)^{#upper} (s - m.v)_+^3 / (6 m1 m2 m3)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        m = rng.integers(-7, 8, size=3)
        m[m == 0] = 3
        lo = sum(min(0, x) for x in m)
        hi = sum(max(0, x) for x in m)
        s = Q(int(rng.integers(0, 64)), 64) * (hi - lo) + lo
        exact = X.truncated_box_volume(m, s)
        got = oracle_mod.clip_volume(CUBE_V, CUBE_F, [list(m) + [float(s)]])
        assert abs(got - float(exact)) <= 1e-15, (m, s, got, exact)


def test_clip_degenerate_planes(oracle_mod):
    """Planes through faces, edges and vertices: closed half-spaces."""
    cases = [([1, 0, 0, 1.0], 1.0), ([1, 0, 0, 0.0], 0.0), ([-1, 0, 0, 0.0], 1.0),
             ([1, 1, 0, 1.0], 0.5), ([1, 1, 1, 0.0], 0.0), ([1, 1, 1, 3.0], 1.0),
             ([0, 0, 1, 0.5], 0.5)]
    for pl, v in cases:
        assert oracle_mod.clip_volume(CUBE_V, CUBE_F, [pl]) == pytest.approx(v, abs=1e-15)


def test_clip_tet_halfspace_divided_differences(oracle_mod):
    """|T ∩ {n.x <= s}| / |T| = sum_i (s - h_i)_+^3 / prod_{j!=i} (h_j - h_i)
    with h_i = n.v_i distinct (the B-spline / divided-difference form)."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        T = rng.random((4, 3))
        if np.linalg.det(T[1:] - T[0]) < 0:
            T[[1, 2]] = T[[2, 1]]
        n = rng.normal(size=3)
        h = T @ n
        s = rng.uniform(h.min(), h.max())
        frac = 0.0
        for i in range(4):
            den = np.prod([h[j] - h[i] for j in range(4) if j != i])
            frac += max(0.0, s - h[i]) ** 3 / den
        vol = abs(np.linalg.det(T[1:] - T[0])) / 6
        got = oracle_mod.clip_volume(T, TET_F, [list(n) + [s]])
        assert got == pytest.approx(frac * vol, rel=1e-9, abs=1e-15)


def test_clip_tet_by_box_exact_rational(oracle_mod):
    """Tet ∩ box on dyadic data against the exact rational tet-splitting clipper."""
    rng = np.random.default_rng(3)
    for _ in range(60):
        T = rng.integers(-8, 24, size=(4, 3)) / 16.0
        d = np.linalg.det(T[1:] - T[0])
        if d == 0:
            continue
        if d < 0:
            T[[1, 2]] = T[[2, 1]]
        lo = rng.integers(0, 8, size=3) / 16.0
        hi = lo + rng.integers(2, 12, size=3) / 16.0
        planes = X.box_planes(lo, hi)
        exact = X.tet_halfspaces_volume(T, planes)
        got = oracle_mod.clip_volume(T, TET_F, planes)
        assert abs(got - float(exact)) <= 1e-15 * max(1.0, float(exact)), (T, lo, hi)
        # and with an extra oblique plane
        pl = [int(x) for x in rng.integers(-3, 4, size=3)] + [float(rng.integers(-8, 24) / 16.0)]
        if any(pl[:3]):
            exact2 = X.tet_halfspaces_volume(T, planes + [pl])
            got2 = oracle_mod.clip_volume(T, TET_F, planes + [pl])
            assert abs(got2 - float(exact2)) <= 1e-15, (T, lo, hi, pl)


# --------------------------------------------------------------------------
# mesh geometry and IDW (Section 2, eqs. 2.6-2.7)
# --------------------------------------------------------------------------

def test_geometry_boxes_and_tets(oracle_mod):
    m = W.hex_mesh(3, 4, 5, (0, 0, 0), (1.5, 1.0, 0.5))
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    assert np.allclose(V, (1.5 / 3) * (1.0 / 4) * (0.5 / 5), rtol=1e-14)
    assert np.allclose(xc, 0.5 * (m.cell_lo + m.cell_hi), atol=1e-15)
    t = W.kuhn_tet_mesh(3, 0.2, 7)
    ot = oracle_mod.Oracle(t)
    V, xc, S, cf = ot.geometry()
    P = t.points[t.cell_verts]
    vol = np.einsum("ij,ij->i", P[:, 1] - P[:, 0],
                    np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0])) / 6
    assert (vol > 0).all()
    assert np.allclose(V, vol, rtol=1e-12)
    assert np.allclose(xc, P.mean(1), atol=1e-14)
    assert V.sum() == pytest.approx(1.0, rel=1e-13)
    # closed cells: sum of signed outward area vectors vanishes
    acc = np.zeros((t.n_cells, 3))
    np.add.at(acc, t.owner, S)
    np.add.at(acc, t.neighbour, -S[:t.n_internal])
    assert np.abs(acc).max() < 1e-15
    # owner -> neighbour orientation
    d = xc[t.neighbour] - xc[t.owner[:t.n_internal]]
    assert ((d * S[:t.n_internal]).sum(1) > 0).all()


def test_idw_constant_and_symmetric(oracle_mod):
    m = W.hex_mesh(4, 4, 4)
    o = oracle_mod.Oracle(m)
    Up = o.set_velocity(np.tile([0.3, -1.25, 2.0], (m.n_cells, 1)), np.zeros(m.n_faces))
    assert np.abs(Up - [0.3, -1.25, 2.0]).max() <= 4 * 2.0 * np.finfo(float).eps
    # interior point of a uniform grid: 8 equidistant cells, linear field exact
    V, xc, S, cf = o.geometry()
    phi = 0.7 + xc @ np.array([1.0, -2.0, 0.5])
    pv = o.point_values(phi)
    interior = np.all((m.points > 1e-9) & (m.points < 1 - 1e-9), axis=1)
    exact = 0.7 + m.points @ np.array([1.0, -2.0, 0.5])
    assert np.abs(pv[interior] - exact[interior]).max() < 1e-14


def test_nag_exact_for_linear_fields(oracle_mod):
    """Eqs. 2.6-2.12 reproduce the gradient of a linear field on uniform-hex
    cells whose points are all interior (symmetric IDW, centroid face values)."""
    m = W.hex_mesh(6, 6, 6)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    g = np.array([0.3, -1.7, 2.2])
    phi = 0.1 + xc @ g
    G = o.nag_gradient(phi)
    inner = np.all((m.cell_lo > 1e-9) & (m.cell_hi < 1 - 1e-9), axis=1)
    assert np.abs(G[inner] - g).max() < 1e-12


@pytest.mark.parametrize("meshkind", ["hex", "tets"])
def test_lsq_gradient_exact_for_linear_fields(oracle_mod, meshkind):
    """The generalized LSQ gradient has zero residual for a linear field on
    any mesh, boundary cells and jittered tets included."""
    m = W.hex_mesh(5, 4, 6) if meshkind == "hex" else W.kuhn_tet_mesh(4, 0.2, 7)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    g = np.array([0.3, -1.7, 2.2])
    G = o.lsq_gradient(0.1 + xc @ g)
    assert np.abs(G - g).max() < 1e-12


def test_lsq_gradient_is_the_weighted_least_squares_solution(oracle_mod):
    """Against numpy's SVD least squares on the weighted system, with the
    point-neighbour stencil built here from the cells' vertex lists."""
    m = W.kuhn_tet_mesh(3, 0.2, 11)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    rng = np.random.default_rng(4)
    phi = rng.random(m.n_cells)
    G = o.lsq_gradient(phi)
    cells_of_point = [[] for _ in range(m.n_points)]
    for c, verts in enumerate(m.cell_verts):
        for p in verts:
            cells_of_point[p].append(c)
    for c in range(m.n_cells):
        nb = sorted({k for p in m.cell_verts[c] for k in cells_of_point[p]} - {c})
        D = xc[nb] - xc[c]
        w = 1.0 / np.linalg.norm(D, axis=1)
        sol = np.linalg.lstsq(w[:, None] * D, w * (phi[nb] - phi[c]), rcond=None)[0]
        assert np.abs(G[c] - sol).max() <= 1e-11 * max(1.0, np.abs(sol).max())


# --------------------------------------------------------------------------
# flux polyhedra (eqs. 2.16-2.19) and flux correction (Section 2.3)
# --------------------------------------------------------------------------

def test_uniform_translation_prism(oracle_mod):
    """Uniform translation sweeps exact prisms: V_f(lam) = lam dt U.S_f."""
    t = W.kuhn_tet_mesh(3, 0.2, 11)
    o = oracle_mod.Oracle(t)
    V, xc, S, cf = o.geometry()
    U = np.array([0.4, -0.9, 0.25])
    o.set_point_velocity(np.tile(U, (t.n_points, 1)), S @ U)
    for f in range(0, t.n_faces, 7):
        for lam in (0.3, 1.0, 1.7):
            v = o.flux_volume(f, 0.01, 1.0, lam)
            assert v == pytest.approx(lam * 0.01 * (U @ S[f]), rel=1e-12, abs=1e-18)


def _cube_dilation(oracle_mod, kappa):
    m = W.hex_mesh(1, 1, 1)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    Up = (m.points - xc[0])     # delta_p = -kappa (x_p - x_c) with dt = kappa
    return m, o, Up


def test_dilation_identity(oracle_mod):
    """delta_p = -kappa (x_p - x_c) on one cube: sum_f V_f(lam) =
    V_c (1 - (1 - lam kappa)^3), each face a sixth by symmetry."""
    kappa = 0.37
    m, o, Up = _cube_dilation(oracle_mod, kappa)
    o.set_point_velocity(Up, np.zeros(m.n_faces))
    for lam in (0.1, 0.5, 1.0, 1.9):
        vols = [o.flux_volume(f, kappa, 1.0, lam) for f in range(6)]
        exact = 1.0 - (1.0 - lam * kappa) ** 3
        assert sum(vols) == pytest.approx(exact, rel=1e-14)
        assert np.allclose(vols, exact / 6, rtol=1e-13)


def test_dilation_correction_closed_form_root(oracle_mod):
    """Corrected lam for a prescribed face flux: V/6 (1 - (1 - lam k)^3) = F dt,
    so lam = (1 - (1 - 6 F dt / V)^(1/3)) / k."""
    kappa = 0.2
    m, o, Up = _cube_dilation(oracle_mod, kappa)
    Fdt = np.array([0.01, 0.02, 0.05, 0.08, 0.03, 0.001])
    dt = kappa
    o.set_point_velocity(Up, Fdt / dt)
    lam, it, st, bad = o.flux_correction(dt, 1.0)
    exact = (1 - (1 - 6 * Fdt) ** (1 / 3)) / kappa
    assert bad == 0
    assert np.allclose(lam, exact, rtol=1e-13)


def test_discrete_reynolds_identity(oracle_mod):
    """At lam = 1, sum_f sgn_cf V_f = V_c - |backtracked cell|; the swept
    sides cancel between neighbouring faces.  The backtracked cell's volume
    is taken here from its fan-triangulated faces (about the mean of each
    face's swept points) by the divergence theorem."""
    t = W.kuhn_tet_mesh(2, 0.2, 5)
    o = oracle_mod.Oracle(t)
    V, xc, S, cf = o.geometry()
    rng = np.random.default_rng(9)
    Up = rng.normal(scale=0.05, size=(t.n_points, 3))
    o.set_point_velocity(Up, np.ones(t.n_faces))
    dt = 1.0
    q = t.points - dt * Up
    vf = np.array([o.flux_volume(f, dt, 1.0, 1.0) for f in range(t.n_faces)])
    net = np.zeros(t.n_cells)
    np.add.at(net, t.owner, vf)
    np.add.at(net, t.neighbour, -vf[:t.n_internal])
    back = np.zeros(t.n_cells)
    for f in range(t.n_faces):
        ids = t.face_points[t.face_offsets[f]:t.face_offsets[f + 1]]
        cq = q[ids].mean(0)
        contrib = 0.0
        for i in range(len(ids)):
            a, b = q[ids[i]], q[ids[(i + 1) % len(ids)]]
            contrib += np.dot(cq, np.cross(a, b)) / 6
        back[t.owner[f]] += contrib
        if f < t.n_internal:
            back[t.neighbour[f]] -= contrib
    assert np.abs(net - (V - back)).max() < 1e-15


def _perturbed_sweep(oracle_mod, radius, seed):
    m = W.hex_mesh(5, 5, 5)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    rng = np.random.default_rng(seed)
    U = np.array([0.5, 0.4, 0.3])
    h = 1.0 / 5
    dt = 0.5 * h / np.abs(U).max()
    d = rng.normal(size=(m.n_points, 3))
    d *= (rng.random((m.n_points, 1)) ** (1 / 3)) / np.linalg.norm(d, axis=1)[:, None]
    Up = U + d * radius * h / dt        # swept points moved within a ball
    F0 = S @ U
    o.set_point_velocity(Up, F0)
    lam, it, st, bad = o.flux_correction(dt, 1.0)
    res = np.array([abs(o.flux_volume(f, dt, 1.0, lam[f]) - F0[f] * dt) / abs(F0[f] * dt)
                    for f in range(m.n_faces)])
    for f in np.flatnonzero(st == 1):
        # at the branch extremum, or at the plain sweep when that is nearer
        v = [abs(o.flux_volume(f, dt, 1.0, lam[f] * (1 + e))) for e in (-1e-4, 0.0, 1e-4)]
        at_extremum = v[1] >= max(v[0], v[2])
        assert (at_extremum or abs(abs(lam[f]) - 1.0) < 1e-15) and v[1] < abs(F0[f] * dt)
    return F0, lam, it, st, bad, res


def test_correction_robust_to_perturbation(oracle_mod):
    """Swept points perturbed randomly (Section 2.3 tests up to 20 % of the face
    length) at Co 0.5.  Up to a ball of radius h/(5 sqrt 3) every face converges
    to machine tolerance in 3-5 secant iterations on average, as the paper
    reports; at radius h/5 the few faces whose swept face collapses cannot
    reach the target on the monotone branch and are flagged (status 1), while
    all others still converge."""
    for seed in range(2):
        F0, lam, it, st, bad, res = _perturbed_sweep(oracle_mod, 0.2 / np.sqrt(3), seed)
        assert bad == 0
        assert res[F0 != 0].max() < 1e-13
        assert 3 <= it[F0 != 0].mean() <= 5
        F0, lam, it, st, bad, res = _perturbed_sweep(oracle_mod, 0.2, seed)
        ok = (F0 != 0) & (st == 0)
        assert bad == (st == 1).sum() and bad < 0.02 * (F0 != 0).sum()
        assert res[ok].max() < 1e-13
        assert (res[st == 1] > 0).all()


# --------------------------------------------------------------------------
# reconstruction: positioning (Algorithm 1)
# --------------------------------------------------------------------------

def test_positioning_reproduces_alpha_box(oracle_mod):
    """The positioned plane cuts the exact volume fraction: checked with the
    truncated-box closed form in exact arithmetic."""
    m = W.hex_mesh(4, 4, 4)
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(5)
    alpha = rng.uniform(0.001, 0.999, m.n_cells)
    rec = o.reconstruct(alpha)
    h = 0.25
    for c in range(0, m.n_cells, 5):
        if rec["cls"][c] != 1:
            continue
        n = rec["n"][c]
        if np.any(n == 0):
            continue
        frac = X.truncated_box_volume([Q(x) for x in n], Q(rec["s"][c]),
                                      [Q(x) for x in m.cell_lo[c]],
                                      [Q(x) for x in m.cell_hi[c]]) / Q(h) ** 3
        assert abs(float(frac) - alpha[c]) < 1e-13


def test_positioning_tet_closed_form(oracle_mod):
    t = W.kuhn_tet_mesh(2, 0.2, 3)
    o = oracle_mod.Oracle(t)
    V, xc, S, cf = o.geometry()
    rng = np.random.default_rng(6)
    alpha = rng.uniform(0.01, 0.99, t.n_cells)
    rec = o.reconstruct(alpha)
    for c in range(t.n_cells):
        if rec["cls"][c] != 1:
            continue
        P = t.points[t.cell_verts[c]]
        hh = P @ rec["n"][c]
        s = rec["s"][c]
        frac = 0.0
        for i in range(4):
            den = np.prod([hh[j] - hh[i] for j in range(4) if j != i])
            frac += max(0.0, s - hh[i]) ** 3 / den
        assert frac == pytest.approx(alpha[c], abs=1e-9)


def test_axis_aligned_normal_by_symmetry(oracle_mod):
    m = W.hex_mesh(8, 8, 8)
    o = oracle_mod.Oracle(m)
    lo, hi = m.cell_lo[:, 1], m.cell_hi[:, 1]
    alpha = np.clip((np.minimum(hi, 0.4) - lo) / (hi - lo), 0, 1)
    rec = o.reconstruct(alpha)
    sel = rec["cls"] == 1
    assert sel.any()
    assert np.abs(rec["n"][sel] - [0, 1, 0]).max() < 1e-14
    assert np.abs(rec["s"][sel] - 0.4).max() < 1e-14


# --------------------------------------------------------------------------
# phase flux (eqs. 2.22-2.23) and update (eq. 2.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("meshkind", ["hex", "tet"])
def test_partition_of_unity(oracle_mod, meshkind):
    """sum_c |T ∩ C_c| = |T| for tets inside the domain."""
    m = W.hex_mesh(4, 4, 4) if meshkind == "hex" else W.kuhn_tet_mesh(3, 0.2, 8)
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(7)
    for _ in range(10):
        T = 0.2 + 0.6 * rng.random((4, 3))
        vol = abs(np.linalg.det(T[1:] - T[0])) / 6
        tot = sum(o.tet_cell_volume(T, c) for c in range(m.n_cells))
        assert tot == pytest.approx(vol, rel=1e-12, abs=1e-17)


def test_slab_translation_whole_step_closed_form(oracle_mod):
    """An axis-aligned slab moved along its normal stays exact step after step,
    including the empty-inflow and outflow boundaries."""
    w = W.translate_slab(16, 1, a=0.3, b=0.55, U=(0.25, 0.0, 0.0), steps=40)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    a = w.alpha0.copy()
    for k in range(0, 40, 10):
        a, st, _, _ = o.advect(a, w.dt[k:k + 10], w.scale[k:k + 10])
        assert np.abs(a - W.slab_exact(w, k + 10)).max() < 1e-13


def test_diagonal_plane_translation_3d(oracle_mod):
    """Plane x+y+z < c moved along (1,1,1): symmetry makes the NAG normal exact,
    so one step reproduces the exact fractions away from the boundary."""
    n = 10
    m = W.hex_mesh(n, n, n)
    o = oracle_mod.Oracle(m)
    V, xc, S, cf = o.geometry()
    import workloads.fields as Fd
    U = np.array([1.0, 1.0, 1.0]) * 0.3
    F0 = Fd.flux_constant(m, U)
    o.set_velocity(np.tile(U, (m.n_cells, 1)), F0)
    dt = 0.4 / n / 0.3

    def exact(c0):
        out = np.empty(m.n_cells)
        for i in range(m.n_cells):
            out[i] = float(X.truncated_box_volume([1, 1, 1], Q(c0), m.cell_lo[i], m.cell_hi[i])
                           ) * n ** 3
        return out
    c0 = 1.37
    a0 = exact(c0)
    r = o.step(a0, dt, 1.0)
    ex = exact(c0 + 3 * 0.3 * dt)
    inner = np.all((m.cell_lo > 2.5 / n) & (m.cell_hi < 1 - 2.5 / n), axis=1)
    assert np.abs(r["alpha"] - ex)[inner].max() < 1e-13


def test_disc2d_conservation_boundedness(oracle_mod):
    w = W.disc2d()
    o = oracle_mod.Oracle(w.mesh)
    V, _, _, _ = o.geometry()
    o.set_velocity(w.U0c, w.F0)
    a, st, lam, vp = o.advect(w.alpha0, w.dt, w.scale, check_leak=True)
    m0 = (w.alpha0 * V).sum()
    assert abs((a * V).sum() + st["ledger"] - m0) <= 1e-12 * m0
    assert a.min() > -1e-12 and a.max() < 1 + 1e-12
    assert st["max_leak"] < 1e-13
    assert st["max_corr_residual"] < 1e-13
    assert st["n_clip_errors"] == 0


def test_trivial_faces_full_stencil(oracle_mod):
    """A face whose stencil is all full carries exactly F dt; all empty, 0."""
    m = W.hex_mesh(6, 6, 6)
    o = oracle_mod.Oracle(m)
    import workloads.fields as Fd
    U = np.array([0.2, 0.1, -0.1])
    F0 = Fd.flux_constant(m, U)
    o.set_velocity(np.tile(U, (m.n_cells, 1)), F0)
    alpha = np.ones(m.n_cells)
    rec = o.reconstruct(alpha)
    lam, *_ = o.flux_correction(0.1, 1.0)
    ph = o.phase_flux(0.1, 1.0, lam, alpha)
    ni = m.n_internal
    assert np.array_equal(ph["vphase"][:ni], F0[:ni] * 0.1)
    assert (ph["kind"][:ni] == 2).all()
    ph0 = o.phase_flux(0.1, 1.0, lam, np.zeros(m.n_cells))
    o.reconstruct(np.zeros(m.n_cells))
    ph0 = o.phase_flux(0.1, 1.0, lam, np.zeros(m.n_cells))
    assert (ph0["vphase"] == 0).all()
    del rec


def test_clip_face_in_plane_not_doubled(oracle_mod):
    """A plane containing a face of the polytope (repeated, or with rounding
    putting a vertex a hair outside) removes nothing: exact rational check."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        T = rng.integers(0, 5, (4, 3)) / 4.0
        d = np.linalg.det(T[1:] - T[0])
        if abs(d) < 1e-12:
            continue
        if d < 0:
            T[[2, 3]] = T[[3, 2]]
        pl = [int(x) for x in rng.integers(-2, 3, 3)] + [float(rng.integers(0, 5) / 4.0)]
        if not any(pl[:3]):
            continue
        exact = float(X.tet_halfspaces_volume(T, [pl]))
        assert abs(oracle_mod.clip_volume(T, TET_F, [pl, pl]) - exact) <= 1e-15
    # the plane of face (1, 2, 3) of a tet, with one vertex moved 1e-18 outward
    T = np.array([[0.1, 0.2, 0.1], [1.0, 0.1, 0.2], [0.2, 1.1, 0.0], [0.3, 0.2, 0.9]])
    n = np.cross(T[2] - T[1], T[3] - T[1])
    s = n @ T[1]
    T2 = T.copy()
    T2[2] += 1e-18 * n / np.linalg.norm(n)
    vol = abs(np.linalg.det(T[1:] - T[0])) / 6
    for P in (T, T2):
        assert oracle_mod.clip_volume(P, TET_F, [list(n) + [s]]) == pytest.approx(vol, rel=1e-14)
        assert oracle_mod.clip_volume(P, TET_F, [list(n) + [s]] * 3) == pytest.approx(vol, rel=1e-14)


# --------------------------------------------------------------------------
# reconstruction error E_vsd against an analytic sphere (Section 4.1)
# --------------------------------------------------------------------------

def test_vsd_quadrature_components(oracle_mod):
    """The E_vsd integrator's volumes: |C ∩ ball| against the exact sphere-box
    fractions, and |PLIC polyhedron| against alpha V (the positioning)."""
    from tests.reconstruction_error import _z_lengths, cell_vsd  # noqa: F401
    from workloads import fields
    c, r = np.array([0.5123, 0.4871, 0.5036]), 0.15
    m = W.hex_mesh(12, 12, 12)
    a0 = fields.ball_box_fraction(c, r, m.cell_lo, m.cell_hi)
    o = oracle_mod.Oracle(m)
    rec = o.reconstruct(a0)
    xg, wg = np.polynomial.legendre.leggauss(4)
    for cell in np.flatnonzero(rec["cls"] == 1)[::5]:
        lo, hi = m.cell_lo[cell], m.cell_hi[cell]
        e = np.linspace(0, 1, 17)
        t = (0.5 * (e[:-1, None] + e[1:, None]) + 0.5 * (e[1:, None] - e[:-1, None]) * xg).ravel()
        w = (0.5 * (e[1:, None] - e[:-1, None]) * wg).ravel()
        X, Y = np.meshgrid(lo[0] + t * (hi[0] - lo[0]), lo[1] + t * (hi[1] - lo[1]), indexing="ij")
        Wt = np.outer(w, w) * (hi[0] - lo[0]) * (hi[1] - lo[1])
        V = np.prod(hi - lo)
        I = (Wt * _z_lengths(X, Y, lo[2], hi[2], None, (c, r))).sum()
        R = (Wt * _z_lengths(X, Y, lo[2], hi[2], (rec["n"][cell], rec["s"][cell]), None)).sum()
        assert abs(I - a0[cell] * V) <= 1e-3 * V       # the silhouette slows the rule
        assert abs(R - a0[cell] * V) <= 1e-5 * V


@pytest.mark.slow
def test_vsd_converges_nag_and_lsq(oracle_mod):
    """E_vsd of the sphere reconstruction falls at least threefold from 16^3 to
    32^3 hexahedra with either gradient (second order on coarse meshes,
    Section 4.1.1)."""
    from tests.reconstruction_error import vsd
    from workloads import fields
    c, r = np.array([0.5123, 0.4871, 0.5036]), 0.15
    out = {}
    for n in (16, 32):
        m = W.hex_mesh(n, n, n)
        a0 = fields.ball_box_fraction(c, r, m.cell_lo, m.cell_hi)
        for g in ("nag", "lsq"):
            rec = oracle_mod.Oracle(m, gradient=g).reconstruct(a0)
            out[(n, g)] = vsd(m, rec["cls"], rec["n"], rec["s"], (c, r))
    print("E_vsd", out)
    for g in ("nag", "lsq"):
        assert 0 < out[(32, g)] < out[(16, g)] / 3


# --------------------------------------------------------------------------
# narrow band and wisp redistribution (Section 2.3)
# --------------------------------------------------------------------------

def _cell_points(mesh):
    """Point set of every cell, from the faces (owner and neighbour side)."""
    pts = [set() for _ in range(mesh.n_cells)]
    off = mesh.face_offsets
    for f in range(mesh.n_faces):
        ps = mesh.face_points[off[f]:off[f + 1]]
        pts[mesh.owner[f]].update(ps.tolist())
        if f < mesh.n_internal:
            pts[mesh.neighbour[f]].update(ps.tolist())
    return pts


def _point_neighbours(mesh):
    """Cells other than c sharing a point with c, by brute force over sets."""
    cp = _cell_points(mesh)
    owner_of = {}
    for c, ps in enumerate(cp):
        for p in ps:
            owner_of.setdefault(p, set()).add(c)
    return [sorted(set().union(*(owner_of[p] for p in cp[c])) - {c}) for c in range(mesh.n_cells)]


def test_bulk_cells_are_cells_with_uniform_exact_neighbourhood(oracle_mod):
    """A bulk cell (vanishing gradient): it and every cell sharing a point with
    it hold exactly 0, or all exactly 1.  Brute force over point sets, on a
    field with exact bulk regions, interface cells and wisps (1e-14 and
    1 - 1e-14, which are not exact)."""
    m = W.hex_mesh(12, 6, 6)
    xc = m.cell_centroids()
    a = (xc[:, 0] > 0.5).astype(np.float64)
    a[(np.abs(xc[:, 0] - 0.5) < 0.1) & (xc[:, 1] < 0.4)] = 0.4
    rng = np.random.default_rng(7)
    zero, one = np.flatnonzero(a == 0.0), np.flatnonzero(a == 1.0)
    a[rng.choice(zero, 2, replace=False)] = 1e-14
    a[rng.choice(one, 2, replace=False)] = 1.0 - 1e-14
    nb = _point_neighbours(m)
    expect = np.array([(a[c] in (0.0, 1.0)) and all(a[k] == a[c] for k in nb[c])
                       for c in range(m.n_cells)])
    o = oracle_mod.Oracle(m)
    got = o.bulk_cells(a)
    assert expect.sum() > 10 and (~expect).sum() > 10
    assert np.array_equal(got, expect)


def test_narrow_band_update_is_exact(oracle_mod):
    """Skipping the bulk cells changes nothing in exact arithmetic: their faces
    are all trivial and their net flux is sum_f sgn F_f dt = 0 (eq. 2.4).  One
    step of the deformation field: bulk cells keep their alpha bit for bit,
    every other cell gets the full update, and the full update of a bulk cell
    differs from its alpha only by rounding."""
    w = W.deform3d(16, steps=4)
    full = oracle_mod.Oracle(w.mesh)
    band = oracle_mod.Oracle(w.mesh, band=True)
    for o in (full, band):
        o.set_velocity(w.U0c, w.F0)
    a0 = w.alpha0
    bulk = band.bulk_cells(a0)
    assert bulk.sum() > 0.8 * w.mesh.n_cells
    sf = full.step(a0, w.dt[1], w.scale[1])
    sb = band.step(a0, w.dt[1], w.scale[1])
    assert np.array_equal(sb["alpha"][bulk], a0[bulk])
    assert np.array_equal(sb["alpha"][~bulk], sf["alpha"][~bulk])
    assert np.max(np.abs(sf["alpha"][bulk] - a0[bulk])) < 1e-14
    assert sb["ledger"] == sf["ledger"]


def _chain(alpha):
    """len(alpha) x 1 x 1 hexahedra: cell i shares points with i - 1 and i + 1 only."""
    m = W.hex_mesh(len(alpha), 1, 1)
    return m, np.array(alpha, dtype=np.float64)


def test_wisp_moves_to_receivers_in_proportion_to_room(oracle_mod):
    """A phase wisp between two interface cells moves whole, split in
    proportion to the receivers' room (1 - eps - alpha) V; it ends exactly at 0."""
    eps = Q(1, 10**12)
    m, a = _chain([0.5, 1e-13, 0.3])
    o = oracle_mod.Oracle(m)
    new, cnt = o.redistribute(a)
    mw = Q(a[1])
    r0, r2 = 1 - eps - Q(a[0]), 1 - eps - Q(a[2])
    e0 = Q(a[0]) + mw * r0 / (r0 + r2)
    e2 = Q(a[2]) + mw * r2 / (r0 + r2)
    assert new[1] == 0.0
    assert abs(new[0] - float(e0)) <= 2e-16 * float(e0)
    assert abs(new[2] - float(e2)) <= 2e-16 * float(e2)
    assert cnt == {"wisps": 1, "left": 0, "receivers": 2}


def test_wisp_limited_by_room_keeps_the_rest(oracle_mod):
    """An overshoot larger than the room around it: both receivers are filled
    to 1 - eps and the wisp keeps the remainder."""
    eps = Q(1, 10**12)
    m, a = _chain([0.875, 1.5, 0.9375])
    o = oracle_mod.Oracle(m)
    new, cnt = o.redistribute(a)
    room = (1 - eps - Q(a[0])) + (1 - eps - Q(a[2]))
    assert abs(new[0] - float(1 - eps)) <= 2e-16
    assert abs(new[2] - float(1 - eps)) <= 2e-16
    assert abs(new[1] - float(Q(a[1]) - room)) <= 4e-16
    assert cnt == {"wisps": 1, "left": 1, "receivers": 2}


def test_wisps_share_a_receiver_by_excess(oracle_mod):
    """Two overshoots around one receiver with little room share that room in
    proportion to their excess; a receiver between an overshoot and an
    undershoot takes from one and gives to the other."""
    eps = Q(1, 10**12)
    m, a = _chain([1.0 + 3e-9, 1.0 - 1e-9, 1.0 + 1e-9])
    new, cnt = oracle_mod.Oracle(m).redistribute(a)
    m0, m2 = Q(a[0]) - 1, Q(a[2]) - 1
    room = 1 - eps - Q(a[1])
    assert abs(new[1] - float(1 - eps)) <= 2e-16
    assert abs(new[0] - float(Q(a[0]) - room * m0 / (m0 + m2))) <= 2e-16
    assert abs(new[2] - float(Q(a[2]) - room * m2 / (m0 + m2))) <= 2e-16
    assert cnt["left"] == 2

    m, a = _chain([1.25, 0.5, -0.125])
    new, cnt = oracle_mod.Oracle(m).redistribute(a)
    assert new[0] == 1.0 and new[2] == 0.0
    assert abs(new[1] - 0.625) <= 2e-16
    assert cnt == {"wisps": 2, "left": 0, "receivers": 1}


def test_redistribution_conserves_and_keeps_receivers_in_band(oracle_mod):
    """Along a deformation run with the narrow band and wisps: each pass keeps
    sum V alpha (to rounding), leaves every receiver within [eps, 1 - eps],
    and sets every wisp it moves whole to exactly 0 or 1; over the run the
    total with the boundary ledger is conserved."""
    w = W.deform3d(16, steps=24)
    o = oracle_mod.Oracle(w.mesh, band=True, wisps=True)
    o.set_velocity(w.U0c, w.F0)
    V = o.geometry()[0]
    a = w.alpha0.copy()
    m0 = np.sum(V * a)
    ledger = 0.0
    eps = 1e-12
    total = 0
    for k in range(w.n_steps):
        st = o.step(a, w.dt[k], w.scale[k])
        up, new = st["updated"], st["alpha"]
        ledger += st["ledger"]
        band = (up > eps) & (up < 1 - eps)
        wisp = ~band & (up != 0.0) & (up != 1.0)
        total += wisp.sum()
        assert st["wisp_counts"]["wisps"] == wisp.sum()
        assert abs(np.sum(V * new) - np.sum(V * up)) <= 1e-15 * np.sum(V * up)
        assert np.all(new[band] >= eps * (1 - 1e-12)) and np.all(new[band] <= 1 - eps + 1e-16)
        whole = wisp & ((new == 0.0) | (new == 1.0))
        assert whole.sum() == wisp.sum() - st["wisp_counts"]["left"]
        a = new
    assert total > 100
    assert abs(np.sum(V * a) + ledger - m0) <= 1e-12 * m0


# --------------------------------------------------------------------------
# geometric mapping after refinement (Section 3, Algorithm 2)
# --------------------------------------------------------------------------

def _refined_pair(n, alpha_fn):
    """Uniform n^3 mesh with alpha, and its refinement of the interface cells."""
    from workloads.refine import refine_hex
    m0 = W.hex_mesh(n, n, n)
    a0 = alpha_fn(m0.cell_lo, m0.cell_hi)
    m1, parent, children = refine_hex(n, (a0 > 0) & (a0 < 1))
    return m0, a0, m1, parent, children


def test_mapping_of_a_diagonal_plane_is_exact(oracle_mod):
    """alpha = exact fractions of {x + y + z <= c}: the NAG normal of interior
    cells is (1,1,1)/sqrt 3 by symmetry and the plane is positioned exactly, so
    every child of an interior interface cell gets the exact fraction of the
    half-space in its own box (truncated box in exact rationals).  The parent's
    plane is placed to a fill-level tolerance of 1e-15, which a child of an
    eighth of the volume sees up to eight times over: 1e-14."""
    c = Q(45, 32)
    n = 8

    def frac(lo, hi):
        return np.array([float(X.truncated_box_volume((1, 1, 1), c, tuple(map(Q, l)), tuple(map(Q, h)))
                               / np.prod([Q(b) - Q(a) for a, b in zip(l, h)]))
                         for l, h in zip(lo, hi)])
    m0, a0, m1, parent, _ = _refined_pair(n, frac)
    o0, o1 = oracle_mod.Oracle(m0), oracle_mod.Oracle(m1)
    a1 = o1.map_alpha(o0, a0, np.arange(m1.n_cells + 1), parent)
    exact = frac(m1.cell_lo, m1.cell_hi)
    ijk = np.stack([parent % n, (parent // n) % n, parent // (n * n)], 1)
    interior = np.all((ijk >= 2) & (ijk <= n - 3), axis=1)
    iface = (a0[parent] > 0) & (a0[parent] < 1)
    sel = interior & iface
    assert sel.sum() > 50
    assert np.abs(a1[sel] - exact[sel]).max() < 1e-14
    assert np.array_equal(a1[~iface], a0[parent][~iface])


def test_mapping_conserves_volume_per_parent(oracle_mod):
    """The children of a refined interface cell share exactly the volume its
    PLIC polyhedron held, alpha V (to the positioning tolerance)."""
    from workloads import fields
    n = 10
    m0, a0, m1, parent, (coff, cells) = _refined_pair(
        n, lambda lo, hi: fields.ball_box_fraction((0.52, 0.47, 0.5), 0.27, lo, hi))
    o0, o1 = oracle_mod.Oracle(m0), oracle_mod.Oracle(m1)
    a1 = o1.map_alpha(o0, a0, np.arange(m1.n_cells + 1), parent)
    V0, V1 = o0.geometry()[0], o1.geometry()[0]
    per_parent = np.zeros(m0.n_cells)
    np.add.at(per_parent, parent, a1 * V1)
    assert np.abs(per_parent - a0 * V0).max() <= 2e-15 * V0.max()
    assert np.all((a1 >= -1e-14) & (a1 <= 1 + 1e-14))  # cut volumes round


def test_mapping_back_by_union_restores_alpha(oracle_mod):
    """Refine, then undo it: each uniform cell is the union of its children and
    gets sum alpha V / V back, the original alpha to rounding."""
    from workloads import fields
    n = 8
    m0, a0, m1, parent, (coff, cells) = _refined_pair(
        n, lambda lo, hi: fields.ball_box_fraction((0.5, 0.5, 0.5), 0.3, lo, hi))
    o0, o1 = oracle_mod.Oracle(m0), oracle_mod.Oracle(m1)
    a1 = o1.map_alpha(o0, a0, np.arange(m1.n_cells + 1), parent)
    back = o0.map_alpha(o1, a1, coff, cells)
    assert np.abs(back - a0).max() <= 2e-15
