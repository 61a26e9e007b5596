"""Seeded synthetic unstructured meshes in owner/neighbour face addressing.

Every mesh produced here uses the face-based layout the paper assumes for the
finite-volume method (Section 2): points are stored once, a face is an ordered
list of point indices, and every face has an owner cell; internal faces also
have a neighbour cell with a larger index than the owner, and the point order
of a face makes its area vector (right-hand rule) point out of the owner and
into the neighbour.  Internal faces come first, sorted by (owner, neighbour);
boundary faces follow, sorted by (patch, owner), their area vectors pointing
out of the domain.

This module only builds connectivity and coordinates.  It holds none of the
advection method's arithmetic; the generator keeps what it knows of each
cell's shape (axis-aligned box or tetrahedron vertices) so that initial
volume fractions and cell velocities can be evaluated analytically.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Mesh:
    points: np.ndarray          # (P, 3) float64
    face_offsets: np.ndarray    # (F + 1,) int64
    face_points: np.ndarray     # (sum n_f,) int32
    owner: np.ndarray           # (F,) int32
    neighbour: np.ndarray       # (F_internal,) int32
    n_cells: int
    kind: str                   # "hex" or "tet"
    # generator-side description of the cells (not used by the method)
    cell_lo: Optional[np.ndarray] = None     # hex: (C, 3) lower corner
    cell_hi: Optional[np.ndarray] = None     # hex: (C, 3) upper corner
    cell_verts: Optional[np.ndarray] = None  # tet: (C, 4) point indices
    patch_of_face: Optional[np.ndarray] = None  # (F - F_internal,) int8
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])

    @property
    def n_internal(self) -> int:
        return int(self.neighbour.shape[0])

    def cell_centroids(self) -> np.ndarray:
        """Analytic centroid of each generated cell (box centre, tet vertex mean)."""
        if self.kind == "hex":
            return 0.5 * (self.cell_lo + self.cell_hi)
        return self.points[self.cell_verts].mean(axis=1)

    def face_sizes(self) -> np.ndarray:
        return np.diff(self.face_offsets)


def _finish(points, faces_int, own_int, nei_int, faces_bnd, own_bnd, patch_bnd,
            n_cells, kind, **extra) -> Mesh:
    """Sort faces into owner/neighbour order and pack them as CSR."""
    order = np.lexsort((nei_int, own_int))
    faces_int = faces_int[order]
    own_int = own_int[order]
    nei_int = nei_int[order]
    border = np.lexsort((own_bnd, patch_bnd))
    faces_bnd = faces_bnd[border]
    own_bnd = own_bnd[border]
    patch_bnd = patch_bnd[border]
    nv = faces_int.shape[1]
    assert faces_bnd.shape[1] == nv
    fp = np.concatenate([faces_int, faces_bnd]).astype(np.int32).ravel()
    nf = faces_int.shape[0] + faces_bnd.shape[0]
    offs = np.arange(nf + 1, dtype=np.int64) * nv
    return Mesh(points=np.ascontiguousarray(points, dtype=np.float64),
                face_offsets=offs, face_points=np.ascontiguousarray(fp),
                owner=np.concatenate([own_int, own_bnd]).astype(np.int32),
                neighbour=nei_int.astype(np.int32), n_cells=int(n_cells),
                kind=kind, patch_of_face=patch_bnd.astype(np.int8), **extra)


def hex_mesh(nx: int, ny: int, nz: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Mesh:
    """Uniform hexahedral mesh of the box [lo, hi] with nx*ny*nz cells.

    Coordinates are lo + (hi - lo) * i / n, so dyadic sizes give exact points.
    Boundary patches: 0 x-min, 1 x-max, 2 y-min, 3 y-max, 4 z-min, 5 z-max.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    xs = lo[0] + (hi[0] - lo[0]) * (np.arange(nx + 1) / nx)
    ys = lo[1] + (hi[1] - lo[1]) * (np.arange(ny + 1) / ny)
    zs = lo[2] + (hi[2] - lo[2]) * (np.arange(nz + 1) / nz)
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    points = np.stack([xs[I.ravel()], ys[J.ravel()], zs[K.ravel()]], axis=1)

    def pid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    def cid(i, j, k):
        return i + nx * (j + ny * k)

    fi, oi, ni, fb, ob, pb = [], [], [], [], [], []

    # x-normal faces at x = xs[i]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx + 1), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    quad = np.stack([pid(i, j, k), pid(i, j + 1, k), pid(i, j + 1, k + 1), pid(i, j, k + 1)], 1)
    m = (i > 0) & (i < nx)
    fi.append(quad[m]); oi.append(cid(i[m] - 1, j[m], k[m])); ni.append(cid(i[m], j[m], k[m]))
    m = i == 0
    fb.append(quad[m][:, ::-1]); ob.append(cid(i[m], j[m], k[m])); pb.append(np.full(m.sum(), 0))
    m = i == nx
    fb.append(quad[m]); ob.append(cid(i[m] - 1, j[m], k[m])); pb.append(np.full(m.sum(), 1))

    # y-normal faces at y = ys[j]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny + 1), np.arange(nx), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    quad = np.stack([pid(i, j, k), pid(i, j, k + 1), pid(i + 1, j, k + 1), pid(i + 1, j, k)], 1)
    m = (j > 0) & (j < ny)
    fi.append(quad[m]); oi.append(cid(i[m], j[m] - 1, k[m])); ni.append(cid(i[m], j[m], k[m]))
    m = j == 0
    fb.append(quad[m][:, ::-1]); ob.append(cid(i[m], j[m], k[m])); pb.append(np.full(m.sum(), 2))
    m = j == ny
    fb.append(quad[m]); ob.append(cid(i[m], j[m] - 1, k[m])); pb.append(np.full(m.sum(), 3))

    # z-normal faces at z = zs[k]
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny), np.arange(nx), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    quad = np.stack([pid(i, j, k), pid(i + 1, j, k), pid(i + 1, j + 1, k), pid(i, j + 1, k)], 1)
    m = (k > 0) & (k < nz)
    fi.append(quad[m]); oi.append(cid(i[m], j[m], k[m] - 1)); ni.append(cid(i[m], j[m], k[m]))
    m = k == 0
    fb.append(quad[m][:, ::-1]); ob.append(cid(i[m], j[m], k[m])); pb.append(np.full(m.sum(), 4))
    m = k == nz
    fb.append(quad[m]); ob.append(cid(i[m], j[m], k[m] - 1)); pb.append(np.full(m.sum(), 5))

    kc, jc, ic = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell_lo = np.stack([xs[ic.ravel()], ys[jc.ravel()], zs[kc.ravel()]], 1)
    cell_hi = np.stack([xs[ic.ravel() + 1], ys[jc.ravel() + 1], zs[kc.ravel() + 1]], 1)
    return _finish(points, np.concatenate(fi), np.concatenate(oi), np.concatenate(ni),
                   np.concatenate(fb), np.concatenate(ob), np.concatenate(pb),
                   nx * ny * nz, "hex", cell_lo=cell_lo, cell_hi=cell_hi,
                   meta={"nx": nx, "ny": ny, "nz": nz, "lo": lo.tolist(), "hi": hi.tolist()})


def _tet_faces(tets: np.ndarray, n_points: int):
    """Unique triangles of a positively oriented tet mesh, owner/neighbour ordered."""
    a, b, c, d = tets[:, 0], tets[:, 1], tets[:, 2], tets[:, 3]
    nt = tets.shape[0]
    # outward (counter-clockwise seen from outside) faces of a positive tet
    tri = np.stack([np.stack([b, c, d], 1), np.stack([a, d, c], 1),
                    np.stack([a, b, d], 1), np.stack([a, c, b], 1)], 1).reshape(-1, 3)
    tet_of = np.repeat(np.arange(nt, dtype=np.int64), 4)
    s = np.sort(tri, axis=1).astype(np.int64)
    assert n_points < (1 << 21)
    key = (s[:, 0] << 42) | (s[:, 1] << 21) | s[:, 2]
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    first = np.ones(key_s.shape[0], dtype=bool)
    first[1:] = key_s[1:] != key_s[:-1]
    gid = np.cumsum(first) - 1
    counts = np.bincount(gid)
    assert counts.max() <= 2, "non-manifold tet mesh"
    starts = np.flatnonzero(first)
    pair = counts[gid[starts]] == 2
    # internal: instances starts[pair] and starts[pair] + 1 (sorted stably by key,
    # so the first instance has the lower tet id since tet_of is increasing)
    i0 = order[starts[pair]]
    i1 = order[starts[pair] + 1]
    t0, t1 = tet_of[i0], tet_of[i1]
    own = np.minimum(t0, t1)
    nei = np.maximum(t0, t1)
    use = np.where(t0 < t1, i0, i1)
    faces_int = tri[use]
    ib = order[starts[~pair]]
    faces_bnd = tri[ib]
    own_bnd = tet_of[ib]
    return faces_int, own, nei, faces_bnd, own_bnd


def kuhn_tet_mesh(n: int, jitter: float = 0.2, seed: int = 1305) -> Mesh:
    """Jittered Kuhn tetrahedral mesh of the unit cube: n^3 hexes, 6 tets each.

    Lattice points (i, j, k)/n are jittered by a seeded uniform draw in
    [-jitter*h, jitter*h] per coordinate (drawn as an (n+1, n+1, n+1, 3) array in
    C order over (i, j, k, xyz)); a coordinate on a boundary plane is left
    unjittered.  Every hex is split conformingly along its v000-v111 diagonal; the
    odd-permutation tets get two vertices swapped so every tet is positive.
    """
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter * h, jitter * h, size=(n + 1, n + 1, n + 1, 3))
    idx = np.arange(n + 1)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    lattice = np.stack([I, J, K], -1).astype(np.float64) * h
    interior = (np.stack([I, J, K], -1) > 0) & (np.stack([I, J, K], -1) < n)
    lattice = lattice + np.where(interior, jit, 0.0)
    # point index p = i + (n+1)(j + (n+1)k)
    pts = lattice.transpose(2, 1, 0, 3).reshape(-1, 3)

    def pid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)

    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    perms = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]
    parity = [1, 1, 1, -1, -1, -1]
    tets = np.empty((ii.size, 6, 4), dtype=np.int64)
    for t, (perm, par) in enumerate(zip(perms, parity)):
        o = [0, 0, 0]
        v = [pid(ii, jj, kk)]
        for ax in perm[:2]:
            o[ax] += 1
            v.append(pid(ii + o[0], jj + o[1], kk + o[2]))
        v.append(pid(ii + 1, jj + 1, kk + 1))
        if par < 0:
            v[1], v[2] = v[2], v[1]
        tets[:, t, :] = np.stack(v, 1)
    tets = tets.reshape(-1, 4)
    fi, oi, ni, fb, ob = _tet_faces(tets, pts.shape[0])
    pb = np.zeros(fb.shape[0], dtype=np.int64)
    return _finish(pts, fi, oi, ni, fb, ob, pb, tets.shape[0], "tet",
                   cell_verts=tets.astype(np.int32),
                   meta={"n": n, "jitter": jitter, "seed": seed})


def single_cell_mesh(points: np.ndarray, faces: list[list[int]]) -> Mesh:
    """A one-cell mesh from explicit outward-oriented faces (all boundary)."""
    offs = np.zeros(len(faces) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(f) for f in faces])
    return Mesh(points=np.ascontiguousarray(points, dtype=np.float64), face_offsets=offs,
                face_points=np.concatenate([np.asarray(f, dtype=np.int32) for f in faces]),
                owner=np.zeros(len(faces), dtype=np.int32),
                neighbour=np.zeros(0, dtype=np.int32), n_cells=1, kind="poly",
                patch_of_face=np.zeros(len(faces), dtype=np.int8))


def unit_cube_cell(lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Mesh:
    """One hexahedral cell with outward faces (boundary patches as in hex_mesh)."""
    m = hex_mesh(1, 1, 1, lo, hi)
    return m
