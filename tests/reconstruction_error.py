"""Volume of symmetric difference E_vsd (Section 4.1) between the PLIC
polyhedra of the interface cells and an analytic ball, on hexahedral meshes.

The paper measures against a tool mesh; here the true geometry is the ball
itself and every volume is integrated over the cell's x-y footprint (the
"integration approach" of that section): the length of the z-interval inside
the cell, the ball and the plane's phase side {n.x <= s}, by composite
Gauss-Legendre.  E_c = |R_c| + |I_c| - 2 |R_c ∩ I_c| with R_c the PLIC polyhedron
and I_c = C ∩ ball, all three with the same quadrature.  Test harness only."""
from __future__ import annotations

import numpy as np


def _z_lengths(X, Y, z0, z1, plane, ball):
    """Length of {z in [z0, z1]} ∩ plane side ∩ ball at the points (X, Y)."""
    lo = np.full(X.shape, z0, dtype=np.float64)
    hi = np.full(X.shape, z1, dtype=np.float64)
    if ball is not None:
        c, r = ball
        rho2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2
        h = np.sqrt(np.maximum(r * r - rho2, 0.0))
        inside = rho2 < r * r
        lo = np.where(inside, np.maximum(lo, c[2] - h), np.inf)
        hi = np.where(inside, np.minimum(hi, c[2] + h), -np.inf)
    if plane is not None:
        n, s = plane
        t = s - n[0] * X - n[1] * Y
        if n[2] > 0:
            hi = np.minimum(hi, t / n[2])
        elif n[2] < 0:
            lo = np.maximum(lo, t / n[2])
        else:
            hi = np.where(t >= 0, hi, -np.inf)
    return np.maximum(hi - lo, 0.0)


def cell_vsd(lo, hi, plane, ball, panels=16, order=4):
    """E_c for one box cell [lo, hi] with PLIC plane (n, s) and ball (c, r)."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    ex = np.linspace(lo[0], hi[0], panels + 1)
    ey = np.linspace(lo[1], hi[1], panels + 1)
    px = (0.5 * (ex[:-1, None] + ex[1:, None]) + 0.5 * (ex[1:, None] - ex[:-1, None]) * xg).ravel()
    py = (0.5 * (ey[:-1, None] + ey[1:, None]) + 0.5 * (ey[1:, None] - ey[:-1, None]) * xg).ravel()
    wx = (0.5 * (ex[1:, None] - ex[:-1, None]) * wg).ravel()
    wy = (0.5 * (ey[1:, None] - ey[:-1, None]) * wg).ravel()
    X, Y = np.meshgrid(px, py, indexing="ij")
    Wt = np.outer(wx, wy)
    R = (Wt * _z_lengths(X, Y, lo[2], hi[2], plane, None)).sum()
    I = (Wt * _z_lengths(X, Y, lo[2], hi[2], None, ball)).sum()
    RI = (Wt * _z_lengths(X, Y, lo[2], hi[2], plane, ball)).sum()
    return R + I - 2.0 * RI


def vsd(mesh, cls, nrm, s, ball, **kw):
    """Sum of E_c over the interface cells (class 1) of a hex mesh."""
    tot = 0.0
    for c in np.flatnonzero(cls == 1):
        tot += cell_vsd(mesh.cell_lo[c], mesh.cell_hi[c], (nrm[c], s[c]), ball, **kw)
    return tot
