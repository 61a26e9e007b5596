"""Helpers shared by the GPU parity tests: run a workload through the C ABI
and through the oracle on identical inputs."""
from __future__ import annotations

import numpy as np


def gpu_run(vof, ctx, w, steps=None, alpha=None, params=None):
    """Advance `w` on the GPU; returns alpha and the last step's face data."""
    mesh = vof.upload_mesh(ctx, w.mesh)
    if params:
        p = vof.vof_get_params(mesh)
        for k, v in params.items():
            setattr(p, k, v)
        vof.vof_set_params(mesh, p)
    vof.vof_set_alpha(mesh, w.alpha0 if alpha is None else alpha)
    vof.vof_set_velocity(mesh, w.U0c, w.F0)
    n = w.n_steps if steps is None else steps
    vof.vof_advect(mesh, w.dt[:n], w.scale[:n])
    out = {
        "alpha": vof.vof_read_alpha(mesh),
        "lam": vof.vof_read_face(mesh, vof.VOF_FACE_LAMBDA),
        "vphase": vof.vof_read_face(mesh, vof.VOF_FACE_VPHASE),
        "iters": vof.vof_read_face(mesh, vof.VOF_FACE_ITERS),
        "kind": vof.vof_read_face(mesh, vof.VOF_FACE_KIND),
        "status": vof.vof_read_face(mesh, vof.VOF_FACE_STATUS),
        "stats": vof.vof_get_stats(mesh),
    }
    out["cls"], out["n"], out["s"] = vof.vof_read_planes(mesh)
    out["mesh"] = mesh
    return out


def oracle_run(oracle, w, steps=None, alpha=None, check_leak=False, gradient="nag", band=False,
               wisps=False):
    o = oracle.Oracle(w.mesh, gradient=gradient, band=band, wisps=wisps)
    o.set_velocity(w.U0c, w.F0)
    n = w.n_steps if steps is None else steps
    a0 = w.alpha0 if alpha is None else alpha
    a, st, lam, vp = o.advect(a0, w.dt[:n], w.scale[:n], check_leak=check_leak)
    return o, a, st, lam, vp


def swept_scale(w, S, Up, scale_dt):
    """Gross swept volume of each face, |S_f| max_i |s dt U_p_i|: the size of the
    terms whose signed sum is the flux polyhedron volume.  Where the normal
    flux is small against a tangential sweep the net volume is a difference of
    much larger terms, so FP64 evaluations agree only to eps times this."""
    m = w.mesh
    sp = np.linalg.norm(Up, axis=1)[m.face_points]
    n = np.diff(m.face_offsets)
    face_of = np.repeat(np.arange(m.n_faces), n)
    mx = np.zeros(m.n_faces)
    np.maximum.at(mx, face_of, sp)
    return np.linalg.norm(S, axis=1) * mx * abs(scale_dt)


def face_size_floor(w, V):
    """max(V_owner, d_f^3) per face, d_f = twice the largest distance of a face
    point from the face centre.  Each of the flux polyhedron's tetrahedra is
    rounded to a few eps times the product of its edges, which are as long as
    the face however short the sweep: the sum is good to about 1e-14 d_f^3
    (20 eps h^3 on hex faces) even where F dt and the sweep are tiny.  On
    jittered tets d_f^3 exceeds a sliver owner's volume many times over."""
    m = w.mesh
    n = np.diff(m.face_offsets)
    face_of = np.repeat(np.arange(m.n_faces), n)
    P = m.points[m.face_points]
    c = np.zeros((m.n_faces, 3))
    np.add.at(c, face_of, P)
    c /= n[:, None]
    r = np.zeros(m.n_faces)
    np.maximum.at(r, face_of, np.linalg.norm(P - c[face_of], axis=1))
    return np.maximum(V[m.owner], (2.0 * r) ** 3)


def vphase_tolerance(w, V, scale_dt, S=None, Up=None):
    """Per-face bound 1e-12 * max(|F| dt, gross swept volume, 1e-2 max(V_owner, d_f^3)).

    The absolute floor 1e-14 max(V_owner, d_f^3) is the FP64 rounding of the
    polyhedron's tetrahedra, whose edges are as long as the face however small
    the sweep (see face_size_floor)."""
    F = np.abs(w.F0) * abs(scale_dt)
    ref = np.maximum(F, 1e-2 * face_size_floor(w, V))
    if S is not None:
        ref = np.maximum(ref, swept_scale(w, S, Up, scale_dt))
    return 1e-12 * ref
