"""One level of 2:1 refinement of a uniform hexahedral mesh.

Selected cells of the n^3 box mesh are split into eight; the remaining
(coarse) cells keep their shape but take the points that their refined
neighbours add on shared edges, so every face lists every mesh point on its
boundary (faces of up to eight points) and the mesh stays conforming.  A face
between a coarse and a refined cell is one quarter of the coarse cell's side.
This is the topology the paper's hexahedral refinement produces (Section 3);
the module builds connectivity and coordinates only.

Coordinates sit on the lattice of spacing h / 2 (h = 1/n along each axis), so
a coarse cell spans two lattice steps and a fine cell one.
"""
from __future__ import annotations

import numpy as np

from .meshes import Mesh

_MAX_REFINED_SIDES = 3  # 6 + 3 k faces for k refined face neighbours: at most 15


def close_refinement(n: int, mask: np.ndarray) -> np.ndarray:
    """Also refine every coarse cell with more than three refined face
    neighbours, until none is left (so no cell has more than 15 faces)."""
    m = np.asarray(mask, dtype=bool).reshape(n, n, n).copy()  # [k, j, i]
    while True:
        cnt = np.zeros(m.shape, dtype=np.int32)
        for ax in range(3):
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[ax] = slice(0, n - 1)
            sl_hi[ax] = slice(1, n)
            cnt[tuple(sl_lo)] += m[tuple(sl_hi)]
            cnt[tuple(sl_hi)] += m[tuple(sl_lo)]
        add = ~m & (cnt > _MAX_REFINED_SIDES)
        if not add.any():
            return m.ravel()
        m |= add


def refine_hex(n: int, mask, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Refine the cells of the uniform n^3 hex mesh where `mask` (length n^3,
    cell i + n (j + n k)) is true, after `close_refinement`.

    Returns (mesh, parent, children): parent[c] is the cell of the uniform
    mesh that new cell c lies in; children (CSR offsets, cells) lists for
    every uniform cell the new cells it is made of (itself, or its eight
    children).  New cells follow the uniform cells' order, children in
    (z, y, x) order inside their parent."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ref = close_refinement(n, mask)
    N = 2 * n  # lattice cells per axis
    # cells: lattice boxes [b0, b1) per axis (x, y, z)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    nsub = np.where(ref, 8, 1)
    parent = np.repeat(np.arange(n ** 3), nsub)
    coff = np.concatenate([[0], np.cumsum(nsub)]).astype(np.int64)
    nc = int(coff[-1])
    b0 = np.empty((nc, 3), dtype=np.int64)
    size = np.empty(nc, dtype=np.int64)
    base = np.stack([2 * i, 2 * j, 2 * k], 1)
    crs = ~ref
    b0[coff[:-1][crs]] = base[crs]
    size[coff[:-1][crs]] = 2
    sub = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)])  # x fastest
    rf = np.flatnonzero(ref)
    for s in range(8):
        b0[coff[rf] + s] = base[rf] + sub[s]
        size[coff[rf] + s] = 1
    # lattice unit cube -> cell, indexed [x, y, z]
    own3 = np.empty((N, N, N), dtype=np.int64)
    for sz in (1, 2):
        cs = np.flatnonzero(size == sz)
        for dx in range(sz):
            for dy in range(sz):
                for dz in range(sz):
                    own3[b0[cs, 0] + dx, b0[cs, 1] + dy, b0[cs, 2] + dz] = cs
    # active points: corners of some cell
    act = np.zeros((N + 1, N + 1, N + 1), dtype=bool)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                act[b0[:, 0] + dx * size, b0[:, 1] + dy * size, b0[:, 2] + dz * size] = True
    pid = -np.ones(act.shape, dtype=np.int64)
    # numbered with x fastest: nonzero over the [z, y, x] view walks z, y, x
    zi, yi, xi = np.nonzero(act.transpose(2, 1, 0))
    pid[xi, yi, zi] = np.arange(xi.size)
    span = hi - lo
    points = np.stack([lo[0] + span[0] * (xi / N), lo[1] + span[1] * (yi / N),
                       lo[2] + span[2] * (zi / N)], 1)

    faces, owners, neigh, patches = [], [], [], []
    for d in range(3):
        a, b = (d + 1) % 3, (d + 2) % 3
        # unit squares on lattice planes P = 0..N along d, cells on each side
        P, A, B = np.meshgrid(np.arange(N + 1), np.arange(N), np.arange(N), indexing="ij")
        P, A, B = P.ravel(), A.ravel(), B.ravel()

        def cell_at(p, aa, bb):
            idx = [None, None, None]
            idx[d], idx[a], idx[b] = p, aa, bb
            return own3[idx[0], idx[1], idx[2]]

        left = np.full(P.size, -1, dtype=np.int64)
        right = np.full(P.size, -1, dtype=np.int64)
        ml = P > 0
        left[ml] = cell_at(P[ml] - 1, A[ml], B[ml])
        mr = P < N
        right[mr] = cell_at(P[mr], A[mr], B[mr])
        keep = left != right
        P, A, B, left, right = P[keep], A[keep], B[keep], left[keep], right[keep]
        # squares of one face share (left, right); its rectangle is their hull
        key = (left + 1) * (nc + 1) + (right + 1)
        uk, inv = np.unique(key, return_inverse=True)
        a0 = np.full(uk.size, N + 1)
        a1 = np.full(uk.size, -1)
        b0_ = np.full(uk.size, N + 1)
        b1 = np.full(uk.size, -1)
        np.minimum.at(a0, inv, A)
        np.maximum.at(a1, inv, A + 1)
        np.minimum.at(b0_, inv, B)
        np.maximum.at(b1, inv, B + 1)
        pp = np.zeros(uk.size, dtype=np.int64)
        pp[inv] = P
        L = uk // (nc + 1) - 1
        R = uk % (nc + 1) - 1
        for f in range(uk.size):
            ring = _ring(a0[f], a1[f], b0_[f], b1[f])
            pts = []
            for (ua, ub) in ring:
                idx = [0, 0, 0]
                idx[d], idx[a], idx[b] = pp[f], ua, ub
                q = pid[idx[0], idx[1], idx[2]]
                if q >= 0:
                    pts.append(q)
            # ring order gives the +d normal (e_a x e_b = e_d)
            l, r = L[f], R[f]
            if l >= 0 and r >= 0:
                if l < r:
                    faces.append(pts); owners.append(l); neigh.append(r); patches.append(-1)
                else:
                    faces.append(pts[::-1]); owners.append(r); neigh.append(l); patches.append(-1)
            elif r >= 0:   # P = 0: outward normal is -d
                faces.append(pts[::-1]); owners.append(r); neigh.append(-1); patches.append(2 * d)
            else:          # P = N
                faces.append(pts); owners.append(l); neigh.append(-1); patches.append(2 * d + 1)
    owners = np.array(owners)
    neigh = np.array(neigh)
    patches = np.array(patches)
    internal = np.flatnonzero(neigh >= 0)
    internal = internal[np.lexsort((neigh[internal], owners[internal]))]
    boundary = np.flatnonzero(neigh < 0)
    boundary = boundary[np.lexsort((owners[boundary], patches[boundary]))]
    order = np.concatenate([internal, boundary])
    sizes = np.array([len(faces[f]) for f in order], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    fp = np.array([q for f in order for q in faces[f]], dtype=np.int32)
    h = span / N
    cell_lo = lo + b0 * h
    cell_hi = lo + (b0 + size[:, None]) * h
    mesh = Mesh(points=np.ascontiguousarray(points), face_offsets=offs, face_points=fp,
                owner=owners[order].astype(np.int32),
                neighbour=neigh[internal].astype(np.int32), n_cells=nc, kind="hex",
                cell_lo=cell_lo, cell_hi=cell_hi,
                patch_of_face=patches[boundary].astype(np.int8),
                meta={"n": n, "refined": int(ref.sum())})
    return mesh, parent.astype(np.int32), (coff, np.arange(nc, dtype=np.int32))


def _ring(a0, a1, b0, b1):
    """Lattice points on the boundary of the rectangle [a0, a1] x [b0, b1],
    counter-clockwise in (a, b) from (a0, b0)."""
    out = [(x, b0) for x in range(a0, a1)]
    out += [(a1, y) for y in range(b0, b1)]
    out += [(x, b1) for x in range(a1, a0, -1)]
    out += [(a0, y) for y in range(b1, b0, -1)]
    return out
