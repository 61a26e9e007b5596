"""ctypes binding of the CPU oracle (vof_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use this module; the product path never imports
it.  It shares no code with the GPU library.  See vof_oracle.c for the
passages of the paper each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "vof_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        i64 = C.c_int64
        d = C.c_double
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_eps.argtypes = [vp, d]
        L.orc_set_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_geometry.argtypes = [vp, vp, vp, vp, vp]
        L.orc_stencil_size.restype = i64
        L.orc_stencil_size.argtypes = [vp]
        L.orc_stencil.argtypes = [vp, vp, vp]
        L.orc_set_velocity.argtypes = [vp, vp, vp, vp]
        L.orc_flux_volume.restype = d
        L.orc_flux_volume.argtypes = [vp, i64, d, d, d]
        L.orc_flux_correction.restype = i64
        L.orc_flux_correction.argtypes = [vp, d, d, vp, vp, vp]
        L.orc_reconstruct.restype = i64
        L.orc_reconstruct.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.orc_phase_flux.restype = i64
        L.orc_phase_flux.argtypes = [vp, d, d, vp, vp, vp, C.c_int, vp, vp, vp, vp]
        L.orc_update.restype = d
        L.orc_update.argtypes = [vp, vp, vp, vp]
        L.orc_advect.restype = C.c_int
        L.orc_advect.argtypes = [vp, vp, i64, vp, vp, C.c_int, vp, vp, vp]
        L.orc_clip_volume.restype = d
        L.orc_clip_volume.argtypes = [C.c_int, vp, C.c_int, vp, vp, C.c_int, vp]
        L.orc_cell_cut_volume.restype = d
        L.orc_cell_cut_volume.argtypes = [vp, i64, vp, d]
        L.orc_tet_cell_volume.restype = d
        L.orc_tet_cell_volume.argtypes = [vp, vp, i64]
        L.orc_set_planes.argtypes = [vp, vp, vp, vp]
        L.orc_point_values.argtypes = [vp, vp, vp]
        L.orc_nag_gradient.argtypes = [vp, vp, vp]
        L.orc_lsq_gradient.argtypes = [vp, vp, vp]
        L.orc_set_gradient.argtypes = [vp, C.c_int]
        L.orc_set_point_velocity.argtypes = [vp, vp, vp]
        L.orc_reconstruct_subset.argtypes = [vp, vp, i64, vp]
        L.orc_get_planes.argtypes = [vp, vp, vp, vp]
        L.orc_faces_subset.argtypes = [vp, d, d, vp, i64, vp, vp, vp, vp, vp, vp]
        L.orc_set_band.argtypes = [vp, C.c_int]
        L.orc_set_wisps.argtypes = [vp, C.c_int]
        L.orc_bulk_cells.argtypes = [vp, vp, vp]
        L.orc_redistribute.argtypes = [vp, vp, vp]
        L.orc_map_alpha.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OStats(C.Structure):
    _fields_ = [("n_interface", C.c_int64), ("n_geometric", C.c_int64),
                ("n_fallback", C.c_int64), ("n_unreached", C.c_int64),
                ("n_clip_errors", C.c_int64), ("ledger", C.c_double),
                ("max_leak", C.c_double), ("max_corr_residual", C.c_double),
                ("mean_secant_iters", C.c_double), ("n_wisps", C.c_int64),
                ("n_wisps_left", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Oracle:
    """The oracle on one mesh (points, face CSR, owner, neighbour)."""

    def __init__(self, mesh, eps: float = 1e-12, gradient: str = "nag", band: bool = False,
                 wisps: bool = False):
        L = lib()
        self.mesh = mesh
        self._keep = [np.ascontiguousarray(mesh.points, dtype=np.float64),
                      np.ascontiguousarray(mesh.face_offsets, dtype=np.int64),
                      np.ascontiguousarray(mesh.face_points, dtype=np.int32),
                      np.ascontiguousarray(mesh.owner, dtype=np.int32),
                      np.ascontiguousarray(mesh.neighbour, dtype=np.int32)]
        pts, offs, fp, own, nei = self._keep
        self.nc = int(mesh.n_cells)
        self.nf = int(own.shape[0])
        self.np_ = int(pts.shape[0])
        self.ni = int(nei.shape[0])
        self.h = L.orc_create(self.np_, self.nc, self.nf, self.ni, _p(pts), _p(offs), _p(fp),
                              _p(own), _p(nei))
        L.orc_set_eps(self.h, eps)
        self.set_gradient(gradient)
        self.set_band(band)
        self.set_wisps(wisps)

    def set_gradient(self, kind: str):
        """Gradient of the reconstruction: "nag" (Section 2.2.1) or "lsq" (the
        generalized least-squares gradient of the same section)."""
        if kind not in ("nag", "lsq"):
            raise ValueError(kind)
        lib().orc_set_gradient(self.h, 1 if kind == "lsq" else 0)

    def set_band(self, on: bool):
        """Narrow band (Section 2.3): bulk cells are not updated."""
        self.band = bool(on)
        lib().orc_set_band(self.h, int(self.band))

    def set_wisps(self, on: bool):
        """Wisp redistribution after every update (Section 2.3)."""
        self.wisps = bool(on)
        lib().orc_set_wisps(self.h, int(self.wisps))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # geometry -------------------------------------------------------------
    def geometry(self):
        V = np.empty(self.nc)
        xc = np.empty((self.nc, 3))
        S = np.empty((self.nf, 3))
        cf = np.empty((self.nf, 3))
        lib().orc_geometry(self.h, _p(V), _p(xc), _p(S), _p(cf))
        return V, xc, S, cf

    def stencil(self):
        n = lib().orc_stencil_size(self.h)
        off = np.empty(self.nf + 1, dtype=np.int64)
        cells = np.empty(n, dtype=np.int32)
        lib().orc_stencil(self.h, _p(off), _p(cells))
        return off, cells

    # steps ----------------------------------------------------------------
    def set_velocity(self, Uc, F0):
        Uc = np.ascontiguousarray(Uc, dtype=np.float64)
        F0 = np.ascontiguousarray(F0, dtype=np.float64)
        Up = np.empty((self.np_, 3))
        lib().orc_set_velocity(self.h, _p(Uc), _p(F0), _p(Up))
        return Up

    def set_point_velocity(self, Up, F0=None):
        Up = np.ascontiguousarray(Up, dtype=np.float64)
        F0 = None if F0 is None else np.ascontiguousarray(F0, dtype=np.float64)
        lib().orc_set_point_velocity(self.h, _p(Up), _p(F0))

    def flux_volume(self, f, dt, s, lam):
        return lib().orc_flux_volume(self.h, int(f), float(dt), float(s), float(lam))

    def flux_correction(self, dt, s):
        lam = np.empty(self.nf)
        it = np.empty(self.nf, dtype=np.int32)
        st = np.empty(self.nf, dtype=np.int8)
        bad = lib().orc_flux_correction(self.h, float(dt), float(s), _p(lam), _p(it), _p(st))
        return lam, it, st, bad

    def reconstruct(self, alpha):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        cls = np.empty(self.nc, dtype=np.int8)
        grad = np.empty((self.nc, 3))
        n = np.empty((self.nc, 3))
        s = np.empty(self.nc)
        it = np.empty(self.nc, dtype=np.int32)
        lib().orc_reconstruct(self.h, _p(alpha), _p(cls), _p(grad), _p(n), _p(s), _p(it))
        return {"cls": cls, "grad": grad, "n": n, "s": s, "iters": it}

    def set_planes(self, cls, n, s):
        cls = np.ascontiguousarray(cls, dtype=np.int8)
        n = np.ascontiguousarray(n, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        lib().orc_set_planes(self.h, _p(cls), _p(n), _p(s))

    def phase_flux(self, dt, s, lam, alpha, check_leak=False, status=None):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        status = (np.zeros(self.nf, dtype=np.int8) if status is None
                  else np.ascontiguousarray(status, dtype=np.int8))
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        vp = np.empty(self.nf)
        kind = np.empty(self.nf, dtype=np.int8)
        leak = C.c_double(0.0)
        ne = C.c_int64(0)
        ngeo = lib().orc_phase_flux(self.h, float(dt), float(s), _p(lam), _p(status), _p(alpha),
                                    int(check_leak), _p(vp), _p(kind), C.byref(leak),
                                    C.byref(ne))
        return {"vphase": vp, "kind": kind, "n_geometric": ngeo, "max_leak": leak.value,
                "clip_errors": ne.value}

    def update(self, alpha, vphase):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        vphase = np.ascontiguousarray(vphase, dtype=np.float64)
        out = np.empty(self.nc)
        B = lib().orc_update(self.h, _p(alpha), _p(vphase), _p(out))
        return out, B

    def step(self, alpha, dt, s, check_leak=False):
        """One full step of the path; returns every intermediate."""
        rec = self.reconstruct(alpha)
        lam, it, st, bad = self.flux_correction(dt, s)
        ph = self.phase_flux(dt, s, lam, alpha, check_leak, status=st)
        new, B = self.update(alpha, ph["vphase"])
        out = {"lam": lam, "iters": it, "status": st, "unreached": bad, **ph, "rec": rec}
        if self.wisps:
            out["updated"] = new.copy()
            new, out["wisp_counts"] = self.redistribute(new)
        return {"alpha": new, "ledger": B, **out}

    def bulk_cells(self, alpha):
        """Cells left alone by the narrow band for this alpha (bool per cell)."""
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        out = np.empty(self.nc, dtype=np.int8)
        lib().orc_bulk_cells(self.h, _p(alpha), _p(out))
        return out.astype(bool)

    def redistribute(self, alpha):
        """One wisp redistribution pass; returns the new alpha and the counts
        (wisps, wisps left with a remainder, receivers)."""
        a = np.array(alpha, dtype=np.float64, copy=True)
        cnt = np.zeros(3, dtype=np.int64)
        lib().orc_redistribute(self.h, _p(a), _p(cnt))
        return a, {"wisps": int(cnt[0]), "left": int(cnt[1]), "receivers": int(cnt[2])}

    def advect(self, alpha, dt, scale, check_leak=False):
        a = np.array(alpha, dtype=np.float64, copy=True)
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        scale = np.ascontiguousarray(scale, dtype=np.float64)
        st = OStats()
        lam = np.empty(self.nf)
        vp = np.empty(self.nf)
        lib().orc_advect(self.h, _p(a), int(dt.shape[0]), _p(dt), _p(scale), int(check_leak),
                         C.byref(st), _p(lam), _p(vp))
        return a, st.as_dict(), lam, vp

    def map_alpha(self, src, alpha_src, map_offsets, map_cells):
        """Volume fraction on this mesh from alpha_src on the mesh of the
        oracle `src` (Section 3, Algorithm 2): src reconstructs alpha_src, and
        new cell c takes the old cells map_cells[map_offsets[c]:map_offsets[c+1]]
        (one old cell containing c, or several whose union is c)."""
        alpha_src = np.ascontiguousarray(alpha_src, dtype=np.float64)
        rec = src.reconstruct(alpha_src)
        V_src = src.geometry()[0]
        off = np.ascontiguousarray(map_offsets, dtype=np.int64)
        cells = np.ascontiguousarray(map_cells, dtype=np.int32)
        assert off.shape[0] == self.nc + 1 and off[-1] == cells.shape[0]
        cls = np.ascontiguousarray(rec["cls"], dtype=np.int8)
        n = np.ascontiguousarray(rec["n"], dtype=np.float64)
        s = np.ascontiguousarray(rec["s"], dtype=np.float64)
        out = np.empty(self.nc)
        lib().orc_map_alpha(self.h, _p(off), _p(cells), _p(alpha_src), _p(V_src), _p(cls),
                            _p(n), _p(s), _p(out))
        return out

    # subsets (sampled checks of large runs) --------------------------------
    def reconstruct_subset(self, alpha, cells):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        lib().orc_reconstruct_subset(self.h, _p(alpha), cells.shape[0], _p(cells))
        cls = np.empty(self.nc, dtype=np.int8)
        n = np.empty((self.nc, 3))
        s = np.empty(self.nc)
        lib().orc_get_planes(self.h, _p(cls), _p(n), _p(s))
        return {"cls": cls, "n": n, "s": s}

    def faces_subset(self, dt, s, alpha, faces):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        faces = np.ascontiguousarray(faces, dtype=np.int64)
        k = faces.shape[0]
        lam = np.empty(k)
        it = np.empty(k, dtype=np.int32)
        st = np.empty(k, dtype=np.int8)
        vp = np.empty(k)
        kind = np.empty(k, dtype=np.int8)
        lib().orc_faces_subset(self.h, float(dt), float(s), _p(alpha), k, _p(faces), _p(lam),
                               _p(it), _p(st), _p(vp), _p(kind))
        return {"lam": lam, "iters": it, "status": st, "vphase": vp, "kind": kind}

    # primitives -----------------------------------------------------------
    def cell_cut_volume(self, c, n, s):
        n = np.ascontiguousarray(n, dtype=np.float64)
        return lib().orc_cell_cut_volume(self.h, int(c), _p(n), float(s))

    def tet_cell_volume(self, tet, cell):
        tet = np.ascontiguousarray(tet, dtype=np.float64).reshape(4, 3)
        return lib().orc_tet_cell_volume(self.h, _p(tet), int(cell))

    def point_values(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        out = np.empty(self.np_)
        lib().orc_point_values(self.h, _p(phi), _p(out))
        return out

    def nag_gradient(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        g = np.empty((self.nc, 3))
        lib().orc_nag_gradient(self.h, _p(phi), _p(g))
        return g

    def lsq_gradient(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        g = np.empty((self.nc, 3))
        lib().orc_lsq_gradient(self.h, _p(phi), _p(g))
        return g


def set_threads(n: int) -> int:
    """OpenMP threads of later oracle calls; returns the number before."""
    return int(lib().orc_set_threads(int(n)))


def clip_volume(verts, faces, planes):
    """Volume of a convex polyhedron (outward CCW faces) ∩ {n.x <= s} for each
    plane row (nx, ny, nz, s)."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    offs = np.zeros(len(faces) + 1, dtype=np.int32)
    offs[1:] = np.cumsum([len(f) for f in faces])
    idx = np.ascontiguousarray(np.concatenate([np.asarray(f) for f in faces]), dtype=np.int32)
    planes = np.ascontiguousarray(np.atleast_2d(planes), dtype=np.float64)
    return lib().orc_clip_volume(verts.shape[0], _p(verts), len(faces), _p(offs), _p(idx),
                                 planes.shape[0], _p(planes))
