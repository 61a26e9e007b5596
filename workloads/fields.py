"""Analytic inputs: initial volume fractions, cell velocities, face fluxes.

The paper takes the face volumetric flux from a pressure solve and requires it
to be discretely divergence free (Section 2, eq. 2.4).  For prescribed-velocity
tests we build every face flux as the circulation of a vector potential A with
curl A = U around the face's edge loop (Stokes), computing each mesh edge's
line integral once in a canonical direction and negating it for the reverse
direction.  Every cell's signed face-flux sum then cancels edge by edge, so
eq. 2.4 holds to round-off.

Initial volume fractions are exact cell fractions of a disc, a sphere or a
slotted sphere (the paper sets them by intersecting with a tool mesh, Section
4.1, which is not reproduced here).  None of this is the advection method's
arithmetic; it only prepares its inputs.
"""
from __future__ import annotations

import numpy as np

from .meshes import Mesh

# ----------------------------------------------------------------------------
# exact areas: disc  ∩  axis-aligned rectangle
# ----------------------------------------------------------------------------


def _W(y, rho):
    """∫_0^y sqrt(rho^2 - t^2) dt, with y clipped to [-rho, rho]."""
    with np.errstate(invalid="ignore", divide="ignore"):
        yc = np.clip(y, -rho, rho)
        r = np.where(rho > 0, rho, 1.0)
        root = np.sqrt(np.maximum(rho * rho - yc * yc, 0.0))
        val = 0.5 * (yc * root + rho * rho * np.arcsin(np.clip(yc / r, -1.0, 1.0)))
    return np.where(rho > 0, val, 0.0)


def _quadrant_area(u, v, rho):
    """Area of {y >= u, z >= v} inside the origin-centred disc of radius rho."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), np.broadcast(u, v, rho).shape)
    u, v = np.broadcast_arrays(u, v)
    ystar = np.sqrt(np.maximum(rho * rho - v * v, 0.0))
    ystar = np.where(np.abs(v) < rho, ystar, 0.0)
    a = np.maximum(u, -rho)
    # v >= 0: strip |y| < y*, length w - v
    lo = np.maximum(a, -ystar)
    pos = np.where((v < rho) & (lo < ystar),
                   (_W(ystar, rho) - _W(lo, rho)) - v * (ystar - lo), 0.0)
    # v < 0: length 2w outside |y| < y*, w - v inside
    i1 = np.where(a < -ystar, 2.0 * (_W(-ystar, rho) - _W(a, rho)), 0.0)
    m = np.maximum(a, -ystar)
    i2 = np.where(m < ystar, (_W(ystar, rho) - _W(m, rho)) - v * (ystar - m), 0.0)
    m3 = np.maximum(a, ystar)
    i3 = np.where(m3 < rho, 2.0 * (_W(rho, rho) - _W(m3, rho)), 0.0)
    neg = i1 + i2 + i3
    out = np.where(v >= 0, pos, neg)
    return np.where((a >= rho) | (rho <= 0), 0.0, out)


def disc_rect_area(a, b, rho, y0, y1, z0, z1):
    """Exact area of the disc (centre (a, b), radius rho) inside [y0,y1]x[z0,z1]."""
    return (_quadrant_area(y0 - a, z0 - b, rho) - _quadrant_area(y1 - a, z0 - b, rho)
            - _quadrant_area(y0 - a, z1 - b, rho) + _quadrant_area(y1 - a, z1 - b, rho))


# ----------------------------------------------------------------------------
# sphere ∩ box by x-integration of exact disc-rectangle areas
# ----------------------------------------------------------------------------

_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def sphere_box_volume(c, r, lo, hi):
    """Volume of the ball (centre c, radius r) inside boxes [lo_i, hi_i].

    The section area A(x) is exact; it is integrated over x between the points
    where A is not smooth (the ball's x-extent and the tangencies with the box's
    edge lines and corners), each segment with a smooth-step change of variable
    that removes the square-root endpoint behaviour, then 24-point
    Gauss-Legendre.  Accurate to about 1e-14 of the box volume.
    """
    lo = np.atleast_2d(lo).astype(np.float64)
    hi = np.atleast_2d(hi).astype(np.float64)
    c = np.asarray(c, dtype=np.float64)
    n = lo.shape[0]
    dy = np.stack([lo[:, 1] - c[1], hi[:, 1] - c[1]], 1)
    dz = np.stack([lo[:, 2] - c[2], hi[:, 2] - c[2]], 1)
    dists = np.concatenate([np.abs(dy), np.abs(dz),
                            np.sqrt(dy[:, :, None] ** 2 + dz[:, None, :] ** 2).reshape(n, 4)], 1)
    half = np.sqrt(np.maximum(r * r - dists ** 2, 0.0))
    bps = np.concatenate([c[0] - half, c[0] + half,
                          np.full((n, 1), c[0] - r), np.full((n, 1), c[0] + r)], 1)
    bps = np.clip(bps, lo[:, :1], hi[:, :1])
    bps = np.sort(np.concatenate([lo[:, :1], bps, hi[:, :1]], 1), axis=1)
    a = bps[:, :-1]
    b = bps[:, 1:]
    t = 0.5 * (_GL_X + 1.0)
    w = 0.5 * _GL_W
    phi = t * t * (3.0 - 2.0 * t)
    dphi = 6.0 * t * (1.0 - t)
    x = a[:, :, None] + (b - a)[:, :, None] * phi[None, None, :]
    jac = (b - a)[:, :, None] * dphi[None, None, :] * w[None, None, :]
    rho = np.sqrt(np.maximum(r * r - (x - c[0]) ** 2, 0.0))
    area = disc_rect_area(c[1], c[2], rho,
                          lo[:, 1, None, None], hi[:, 1, None, None],
                          lo[:, 2, None, None], hi[:, 2, None, None])
    return (area * jac).sum(axis=(1, 2))


def ball_box_fraction(c, r, lo, hi, chunk: int = 20000):
    """Volume fraction of each box [lo_i, hi_i] inside the ball."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    vol = np.prod(hi - lo, axis=1)
    near = np.clip(c, lo, hi)
    dmin = np.sqrt(((near - c) ** 2).sum(1))
    far = np.maximum(np.abs(lo - c), np.abs(hi - c))
    dmax = np.sqrt((far ** 2).sum(1))
    out = np.zeros(lo.shape[0])
    out[dmax <= r] = 1.0
    cut = np.flatnonzero((dmin < r) & (dmax > r))
    for s in range(0, cut.size, chunk):
        idx = cut[s:s + chunk]
        out[idx] = sphere_box_volume(c, r, lo[idx], hi[idx]) / vol[idx]
    return np.clip(out, 0.0, 1.0)


def disc_square_fraction(c2, r, lo, hi):
    """Exact fraction of each rectangle [lo,hi] (2-D, extruded) inside a disc."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    area = disc_rect_area(c2[0], c2[1], r, lo[:, 0], hi[:, 0], lo[:, 1], hi[:, 1])
    return np.clip(area / ((hi[:, 0] - lo[:, 0]) * (hi[:, 1] - lo[:, 1])), 0.0, 1.0)


def tet_fraction_sampled(mesh: Mesh, inside, m: int = 12):
    """Approximate fraction of each tet inside the set `inside(x) -> bool`.

    Tets whose four vertices agree are taken as fully in or out (the sets used
    here are much larger than a cell); the others are sampled at m^3 uniformly
    spread points (about 1e-3 of a cell's volume).  Used for slotted-sphere
    starts on tet meshes.
    """
    tv = mesh.points[mesh.cell_verts]                      # (C, 4, 3)
    ins = inside(tv.reshape(-1, 3)).reshape(-1, 4)
    out = ins.all(1).astype(np.float64)
    cut = np.flatnonzero(ins.any(1) & ~ins.all(1))
    # uniform sample of the simplex: midpoints of an m^3 grid of the unit cube,
    # coordinates sorted (a measure-preserving 6-to-1 map onto the simplex)
    g = (np.arange(m) + 0.5) / m
    u = np.sort(np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3), axis=1)
    w4 = np.stack([u[:, 0], u[:, 1] - u[:, 0], u[:, 2] - u[:, 1], 1.0 - u[:, 2]], 1)
    for s in range(0, cut.size, 2048):
        idx = cut[s:s + 2048]
        x = np.einsum("sv,cvd->csd", w4, tv[idx])
        out[idx] = inside(x.reshape(-1, 3)).reshape(len(idx), -1).mean(1)
    return out


# ----------------------------------------------------------------------------
# velocity fields and their vector potentials
# ----------------------------------------------------------------------------


def sinpi(x):
    """sin(pi x), exactly 0 at integer x (so walls and mid-planes get exact zeros)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x == np.round(x), 0.0, np.sin(np.pi * x))


def deformation_velocity(x):
    """Spatial part of the 3-D deformation field (Section 4.2.3, eq. 4.6)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    s = sinpi
    return np.stack([2.0 * s(2 * Y) * s(X) ** 2 * s(2 * Z),
                     -s(2 * X) * s(Y) ** 2 * s(2 * Z),
                     -s(2 * X) * s(2 * Y) * s(Z) ** 2], -1)


def deformation_potential(x):
    """A with curl A = deformation_velocity: (0, -s²πx s2πy s²πz, s²πx s²πy s2πz)/π."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    s = sinpi
    pi = np.pi
    return np.stack([np.zeros_like(X),
                     -s(X) ** 2 * s(2 * Y) * s(Z) ** 2 / pi,
                     s(X) ** 2 * s(Y) ** 2 * s(2 * Z) / pi], -1)


def _edge_integral_gauss(potential, p, q, order: int = 8):
    xg, wg = np.polynomial.legendre.leggauss(order)
    t = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    d = q - p
    acc = np.zeros(p.shape[0])
    for tk, wk in zip(t, w):
        acc += wk * (potential(p + tk * d) * d).sum(-1)
    return acc


def _deformation_edge_integral(p, q):
    """Exact ∮-contribution of a straight edge for axis-aligned edges, else Gauss."""
    d = q - p
    ax = np.abs(d) > 0
    only = ax.sum(1) == 1
    out = _edge_integral_gauss(deformation_potential, p, q)
    s = sinpi
    pi = np.pi
    cos = np.cos
    ye = only & ax[:, 1]
    if ye.any():
        X, Z = p[ye, 0], p[ye, 2]
        out[ye] = (s(X) ** 2 * s(Z) ** 2 / (2 * pi * pi)) * (
            cos(2 * pi * q[ye, 1]) - cos(2 * pi * p[ye, 1]))
    ze = only & ax[:, 2]
    if ze.any():
        X, Y = p[ze, 0], p[ze, 1]
        out[ze] = -(s(X) ** 2 * s(Y) ** 2 / (2 * pi * pi)) * (
            cos(2 * pi * q[ze, 2]) - cos(2 * pi * p[ze, 2]))
    xe = only & ax[:, 0]
    out[xe] = 0.0
    return out


def rotation_velocity(x, omega, origin, axis=(0.0, 0.0, 1.0)):
    """Rigid rotation U = Ω × (x - o), Ω = omega * axis."""
    Om = omega * np.asarray(axis, dtype=np.float64)
    return np.cross(np.broadcast_to(Om, x.shape), x - np.asarray(origin))


def _rotation_edge_integral(p, q, omega, origin, axis=(0.0, 0.0, 1.0)):
    """Exact line integral of A = -|x-o|²Ω/2 along p -> q."""
    Om = omega * np.asarray(axis, dtype=np.float64)
    a = p - origin
    b = q - origin
    return -((q - p) @ Om) * ((a * a).sum(1) + (a * b).sum(1) + (b * b).sum(1)) / 6.0


def _constant_edge_integral(p, q, U):
    """Exact line integral of A = (U × x)/2 along p -> q (curl A = U)."""
    U = np.asarray(U, dtype=np.float64)
    return 0.25 * (np.cross(np.broadcast_to(U, p.shape), p + q) * (q - p)).sum(1)


def shear_velocity(x, u_max: float = 1.0, R: float = 0.5):
    """Spatial part of the shear field (Section 4.2.2, eq. 4.5), read as
    (sin 2πy sin²πx, -sin 2πx sin²πy, u_max (1 - r/R)²), r the distance to the
    axis x = y = 1/2."""
    X, Y = x[..., 0], x[..., 1]
    s = sinpi
    r = np.hypot(X - 0.5, Y - 0.5)
    return np.stack([s(2 * Y) * s(X) ** 2, -s(2 * X) * s(Y) ** 2,
                     u_max * (1.0 - r / R) ** 2], -1)


def _shear_Ay(x, y, u_max: float, R: float):
    """A_y(x, y) = ∫_0^x w(s, y) ds for w = u_max (1 - r/R)², in closed form:
    with t = s - 1/2 and a = y - 1/2, ∫ r dt = (t r + a² asinh(t/|a|)) / 2 and
    ∫ r² dt = t³/3 + a² t."""
    a = y - 0.5
    aa = np.abs(a)

    def F1(t):
        r = np.hypot(t, a)
        safe = np.where(aa > 0, aa, 1.0)
        return 0.5 * (t * r + np.where(aa > 0, a * a * np.arcsinh(t / safe), 0.0))

    def F2(t):
        return t ** 3 / 3.0 + a * a * t

    t1, t0 = x - 0.5, -0.5
    return u_max * (x - 2.0 / R * (F1(t1) - F1(t0)) + (F2(t1) - F2(t0)) / (R * R))


def _shear_edge_integral(p, q, u_max: float = 1.0, R: float = 0.5, order: int = 24):
    """Line integral of A = (0, A_y(x, y), ψ(x, y)), ψ = sin²πx sin²πy / π, along
    axis-aligned edges: z-edges ψ Δz exactly, y-edges ∫ A_y dy by Gauss-Legendre,
    x-edges 0 (curl A = shear_velocity)."""
    d = q - p
    out = np.zeros(p.shape[0])
    ze = np.abs(d[:, 2]) > 0
    s = sinpi
    out[ze] = s(p[ze, 0]) ** 2 * s(p[ze, 1]) ** 2 / np.pi * d[ze, 2]
    ye = np.abs(d[:, 1]) > 0
    if ye.any():
        xg, wg = np.polynomial.legendre.leggauss(order)
        x, y0, y1 = p[ye, 0], p[ye, 1], q[ye, 1]
        acc = np.zeros(x.shape[0])
        for tk, wk in zip(0.5 * (xg + 1.0), 0.5 * wg):
            acc += wk * _shear_Ay(x, y0 + tk * (y1 - y0), u_max, R)
        out[ye] = acc * (y1 - y0)
    if (np.abs(d) > 0).sum(1).max(initial=0) > 1:
        raise ValueError("shear fluxes are defined for axis-aligned (hex) edges")
    return out


def face_flux_from_edges(mesh: Mesh, edge_integral):
    """F_f = Σ over the face's directed edges of ∫ A·dl (edge values shared)."""
    offs = mesh.face_offsets
    fp = mesh.face_points.astype(np.int64)
    n = np.diff(offs)
    face_of = np.repeat(np.arange(mesh.n_faces), n)
    pos = np.arange(fp.size) - offs[face_of]
    nxt = offs[face_of] + (pos + 1) % n[face_of]
    a = fp
    b = fp[nxt]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * mesh.n_points + hi
    ukey, inv = np.unique(key, return_inverse=True)
    ua = ukey // mesh.n_points
    ub = ukey % mesh.n_points
    e = edge_integral(mesh.points[ua], mesh.points[ub])
    sign = np.where(a < b, 1.0, -1.0)
    contrib = sign * e[inv]
    F = np.zeros(mesh.n_faces)
    # fixed-order per-face sums
    np.add.at(F, face_of, contrib)
    return F


def flux_constant(mesh: Mesh, U):
    return face_flux_from_edges(mesh, lambda p, q: _constant_edge_integral(p, q, U))


def flux_deformation(mesh: Mesh):
    return face_flux_from_edges(mesh, _deformation_edge_integral)


def flux_rotation(mesh: Mesh, omega, origin, axis=(0.0, 0.0, 1.0)):
    o = np.asarray(origin, dtype=np.float64)
    return face_flux_from_edges(mesh, lambda p, q: _rotation_edge_integral(p, q, omega, o, axis))


def flux_shear(mesh: Mesh, u_max: float = 1.0, R: float = 0.5):
    return face_flux_from_edges(mesh, lambda p, q: _shear_edge_integral(p, q, u_max, R))
