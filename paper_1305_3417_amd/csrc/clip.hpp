// clip.hpp -- phase volume of one tetrahedron of a flux polyhedron (step 5),
// shared by the clip kernel and host builds of it.
//
// Tetrahedron k of the flux polyhedron of face f at its corrected lam, apex at
// the face centre (local origin):
//   k = 5 i      top    (c_q, q_i+1, q_i)
//   k = 5 i + 1  side   (m_i, p_i+1, p_i)
//   k = 5 i + 2         (m_i, p_i, q_i)
//   k = 5 i + 3         (m_i, q_i, q_i+1)
//   k = 5 i + 4         (m_i, q_i+1, p_i+1)
// Returns its signed volume times the fraction lying in the phase region:
// sum over stencil cells of |T ∩ C_c ∩ H_c| (eqs. 2.22-2.23), H = the PLIC
// half-space in interface cells, all space in full cells, alpha-weighted in
// vanishing-gradient cells, nothing in empty cells.
#pragma once

#include "geom.hpp"
#include "vof_internal.h"

namespace vof {

VHD v3 xyz4(double4 a) { return mk3(a.x, a.y, a.z); }

// Position x and reference velocity u of point q from its 48-byte record.
struct PointRec {
  v3 x, u;
};
VHD PointRec point_rec(const double *XU, int q) {
  const double2 *r = reinterpret_cast<const double2 *>(XU + 6 * (int64_t)q);
  const double2 a = r[0], b = r[1], c = r[2];
  return PointRec{mk3(a.x, a.y, b.x), mk3(b.y, c.x, c.y)};
}

// Bounding box of tet (0, t1, t2, t3) shifted by c.
VHD void tet_bbox(v3 c, v3 t1, v3 t2, v3 t3, v3 &lo, v3 &hi) {
  lo = mk3(dmin(dmin(0.0, t1.x), dmin(t2.x, t3.x)), dmin(dmin(0.0, t1.y), dmin(t2.y, t3.y)),
           dmin(dmin(0.0, t1.z), dmin(t2.z, t3.z))) + c;
  hi = mk3(dmax(dmax(0.0, t1.x), dmax(t2.x, t3.x)), dmax(dmax(0.0, t1.y), dmax(t2.y, t3.y)),
           dmax(dmax(0.0, t1.z), dmax(t2.z, t3.z))) + c;
}

// With check_stencil set, *deficit receives the signed volume of the tet that
// no stencil cell covers (summed over a face it must vanish unless the flux
// polyhedron leaves its stencil) and *gross its unsigned volume.
// Vertices of tetrahedron k of face f's flux polyhedron at its corrected lam,
// relative to the face centre c (the apex is the origin), positively ordered;
// sgn is the orientation of the tet in the signed decomposition.  Returns
// false for k beyond 5n or a flat tet.
VHD bool flux_tet(const DMesh &m, const DState &s, double dt, double sc, int f, int k, v3 &c,
                  v3 &t1, v3 &t2, v3 &t3, double &det, double &sgn) {
  // the padded point list in one or two 16-byte rows, the records loaded
  // together (unrolled, in point order)
  const int32_t *fp = m.fpad + (int64_t)f * m.padw;
  const int4 r0 = *reinterpret_cast<const int4 *>(fp);
  const int4 r1 = m.padw > 4 ? *reinterpret_cast<const int4 *>(fp + 4) : make_int4(-1, -1, -1, -1);
  const int q[kMaxFacePoints] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
  int n = 0;
#pragma unroll
  for (int j = 0; j < kMaxFacePoints; ++j) n += q[j] >= 0;
  if (k >= 5 * n) return false;
  const double sw = -sc * dt * s.lam[f];
  int i = k / 5, type = k - 5 * i;
  int i1 = (i + 1 == n) ? 0 : i + 1;
  c = mk3(0, 0, 0);
  v3 cq = mk3(0, 0, 0);
#pragma unroll
  for (int j = 0; j < kMaxFacePoints; ++j) {
    if (q[j] >= 0) {
      const PointRec pr = point_rec(s.XU, q[j]);
      c = c + pr.x;
      cq = cq + sw * pr.u;
    }
  }
  const PointRec ra = point_rec(s.XU, fp[i]), rb = point_rec(s.XU, fp[i1]);
  v3 pi = ra.x, pj = rb.x;
  v3 qi = sw * ra.u, qj = sw * rb.u;
  c = (1.0 / n) * c;
  pi = pi - c; pj = pj - c;
  qi = pi + qi; qj = pj + qj;
  cq = (1.0 / n) * cq;  // mean sweep; the mean of the face points is the origin
  if (type == 0) { t1 = cq; t2 = qj; t3 = qi; }
  else {
    v3 mi = 0.25 * (pi + pj + qi + qj);
    t1 = mi;
    if (type == 1) { t2 = pj; t3 = pi; }
    else if (type == 2) { t2 = pi; t3 = qi; }
    else if (type == 3) { t2 = qi; t3 = qj; }
    else { t2 = qj; t3 = pj; }
  }
  det = det3(t1, t2, t3);
  if (det == 0.0) return false;
  sgn = det > 0.0 ? 1.0 : -1.0;
  if (det < 0.0) { v3 tmp = t2; t2 = t3; t3 = tmp; det = -det; }
  return true;
}

// Classification of a (tet, cell) pair on the register path: -1 when the
// pair contributes nothing (bounding boxes apart, or the tet outside one of
// the cell's planes), else the number of cell planes that cut the tet, with
// bit j of mask set for plane cf_off[cell] + j (the cell's distinct planes).
VHD int pair_cuts_box(const DMesh &m, v3 c, const Tet &T, v3 lo, v3 hi, v3 blo, v3 bhi, int cell,
                      uint32_t &mask) {
  mask = 0;
  if (hi.x <= blo.x || lo.x >= bhi.x || hi.y <= blo.y || lo.y >= bhi.y || hi.z <= blo.z ||
      lo.z >= bhi.z)
    return -1;
  const int q0 = m.cf_off[cell], q1 = q0 + m.npl[cell];
  for (int q = q0; q < q1; ++q) {
    double4 cp = m.cpl[q];
    v3 nn = xyz4(cp);
    double off = cp.w - dot(nn, c);
    double d1 = off - dot(nn, T.b), d2 = off - dot(nn, T.c), d3 = off - dot(nn, T.d);
    double dmx = dmax(dmax(off, d1), dmax(d2, d3));
    double dmn = dmin(dmin(off, d1), dmin(d2, d3));
    if (dmx <= 0.0) return -1;
    mask |= (dmn < 0.0 ? 1u : 0u) << (q - q0);
  }
  return __builtin_popcount(mask);
}
VHD int pair_cuts(const DMesh &m, v3 c, const Tet &T, v3 lo, v3 hi, int cell, uint32_t &mask) {
  const double4 blo = m.bblo[cell], bhi = m.bbhi[cell];
  return pair_cuts_box(m, c, T, lo, hi, xyz4(blo), xyz4(bhi), cell, mask);
}

// Plane j of a box cell with bounds bb (lo x y z, hi x y z), relative to c:
// j = 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z.
VHD Pl box_plane(const double *bb, int j, v3 c) {
  const int a = j >> 1;
  const double ca = a == 0 ? c.x : (a == 1 ? c.y : c.z);
  const double sg = (j & 1) ? -1.0 : 1.0;
  const double w = (j & 1) ? ca - bb[a] : bb[3 + a] - ca;
  return Pl{a == 0 ? sg : 0.0, a == 1 ? sg : 0.0, a == 2 ? sg : 0.0, w};
}

// The cutting-plane mask of a box cell for the tet (c, c + T.b, c + T.c,
// c + T.d), in box_plane order, or -1 when one plane has the whole tet outside
// (touching included), as pair_cuts_box tests every plane.  Rounding is
// monotone, so the extreme vertex distance to an axis plane is the distance
// of the extreme coordinate.
VHD int box_cuts(const double *bb, v3 c, const Tet &T, uint32_t &mask) {
  mask = 0;
  bool out = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ca = a == 0 ? c.x : (a == 1 ? c.y : c.z);
    const double t1 = a == 0 ? T.b.x : (a == 1 ? T.b.y : T.b.z);
    const double t2 = a == 0 ? T.c.x : (a == 1 ? T.c.y : T.c.z);
    const double t3 = a == 0 ? T.d.x : (a == 1 ? T.d.y : T.d.z);
    const double tmx = dmax(dmax(0.0, t1), dmax(t2, t3));
    const double tmn = dmin(dmin(0.0, t1), dmin(t2, t3));
    const double up = bb[3 + a] - ca;  // +axis: distance up - t
    const double dn = ca - bb[a];      // -axis: distance dn + t
    out |= up - tmn <= 0.0 || dn + tmx <= 0.0;
    mask |= (up - tmx < 0.0 ? 1u : 0u) << (2 * a);
    mask |= (dn + tmn < 0.0 ? 1u : 0u) << (2 * a + 1);
  }
  return out ? -1 : __builtin_popcount(mask);
}

// cell plane q, or the PLIC plane of cell, with its offset relative to c
VHD Pl cell_plane_at(const DMesh &m, int q, v3 c) {
  double4 cp = m.cpl[q];
  v3 nn = xyz4(cp);
  return mkpl(nn, cp.w - dot(nn, c));
}
// cutting plane u of a pair: cell plane u, or plane ~u of a box cell
VHD Pl cut_plane(const DMesh &m, int u, const double *bb, v3 c) {
  return u >= 0 ? cell_plane_at(m, u, c) : box_plane(bb, ~u, c);
}
// a plane (unit normal, offset) relative to the local origin c
VHD Pl plane_rel(double4 pp, v3 c) {
  v3 nn = xyz4(pp);
  return mkpl(nn, pp.w - dot(nn, c));
}
VHD Pl plic_plane_at(const DState &s, int cell, v3 c) { return plane_rel(s.plane[cell], c); }

// The planes bounding the phase region of a classified pair in slots
// p0..p3: the cutting cell planes in mask order, then the PLIC plane of an
// interface cell (slots past the last plane are left unspecified).
VHD void pair_regs_q(const DMesh &m, const DState &s, v3 c, int cell, int cl, int q0,
                     uint32_t mask, Pl &p0, Pl &p1, Pl &p2, Pl &p3) {
  const Pl pl = cl == 1 ? plic_plane_at(s, cell, c) : Pl{0, 0, 0, 0};
  uint32_t mm = mask;
  p0 = mm ? cell_plane_at(m, q0 + __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p1 = mm ? cell_plane_at(m, q0 + __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p2 = mm ? cell_plane_at(m, q0 + __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p3 = mm ? cell_plane_at(m, q0 + __builtin_ctz(mm), c) : pl;
}
VHD void pair_regs(const DMesh &m, const DState &s, v3 c, int cell, int cl, uint32_t mask, Pl &p0,
                   Pl &p1, Pl &p2, Pl &p3) {
  pair_regs_q(m, s, c, cell, cl, m.cf_off[cell], mask, p0, p1, p2, p3);
}

// weight of a covered volume in the phase region of a full (2) or
// vanishing-gradient (3) cell; interface cells carry it in their plane
VHD double class_weight(const DState &s, int cell, int cl) {
  return cl == 3 ? s.alpha[cell] : 1.0;
}

// Register-only phase volume of flux tet k of face f (serial over the
// stencil): every overlapping stencil cell contributes |T ∩ C ∩ H| through
// at most kRegPlanes planes.  Returns false ("deferred") when a pair needs
// more.
VHD bool flux_tet_phase_fast(const DMesh &m, const DState &s, double dt, double sc, int f,
                             int k, double &vol, unsigned long long &npairs) {
  vol = 0.0;
  v3 c, t1, t2, t3;
  double det, sgn;
  if (!flux_tet(m, s, dt, sc, f, k, c, t1, t2, t3, det, sgn)) return true;
  const Tet T{mk3(0, 0, 0), t1, t2, t3};
  v3 lo, hi;
  tet_bbox(c, t1, t2, t3, lo, hi);
  double acc = 0.0;
  unsigned long long np = 0;
  for (int e = m.st_off[f]; e < m.st_off[f + 1]; ++e) {
    const int cell = m.st[e];
    const int cl = s.cls[cell];
    if (cl == 0) continue;
    uint32_t mask;
    const int ncut = pair_cuts(m, c, T, lo, hi, cell, mask);
    if (ncut < 0) continue;
    const int npl = ncut + (cl == 1);
    if (npl > kRegPlanes) return false;
    ++np;
    Pl p0, p1, p2, p3;
    pair_regs(m, s, c, cell, cl, mask, p0, p1, p2, p3);
    acc += class_weight(s, cell, cl) * vol6_planes(T, det, p0, p1, p2, p3, npl);
    if (ncut == 0) break;  // the tet lies inside this cell
  }
  npairs += np;
  vol = sgn * acc / 6.0;
  return true;
}

// Six times the phase volume of the positively ordered flux tet T (apex at
// the origin = face centre c, vol6 = det) inside stencil cell `cell`, with
// (lo, hi) the tet's bounding box in mesh coordinates.  At most three planes
// (cutting cell planes, plus the PLIC plane of an interface cell) take the
// closed forms; more go through the vertex-graph polytope P (only when
// poly_ok; otherwise such a pair returns NaN and is left untouched).  With
// check_stencil, *vcell receives six times |T ∩ C| (the coverage), else 0.
// A pair of four planes handed back: its six-fold phase volume is
// w * det * f4(D), D the 4 x 4 vertex distances written to row[16] (vertex by
// vertex, plane by plane) and f4 the kept fraction of four planes.  With
// `five`, an interface cell's four cutting planes and its PLIC plane: D is
// 4 x 5, in row[20], and f5 the kept fraction of five planes.
struct Four {
  double *row;  // where the distances go
  double w;
  bool on, five;
};
VHD void dists4(const Tet &T, Pl p0, Pl p1, Pl p2, Pl p3, double *row) {
  const Pl pl[4] = {p0, p1, p2, p3};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const D4 d = plane_dists(T, pl[j]);
    row[j] = d.a;
    row[4 + j] = d.b;
    row[8 + j] = d.c;
    row[12 + j] = d.d;
  }
}

VHD void dists5(const Tet &T, Pl p0, Pl p1, Pl p2, Pl p3, Pl p4, double *row) {
  const Pl pl[5] = {p0, p1, p2, p3, p4};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const D4 d = plane_dists(T, pl[j]);
    row[j] = d.a;
    row[5 + j] = d.b;
    row[10 + j] = d.c;
    row[15 + j] = d.d;
  }
}

VHD double pair_phase6(const DMesh &m, const DState &s, const DParams &p, v3 c, const Tet &T,
                       double det, v3 lo, v3 hi, int cell, Poly &P, unsigned long long &ncap,
                       unsigned long long &npairs, double *vcell, bool poly_ok = true,
                       Four *four = nullptr) {
  *vcell = 0.0;
  if (four) four->on = four->five = false;
  const int cl = s.cls[cell];
  if (cl == 0 && !p.check_stencil) return 0.0;
  double4 blo = m.bblo[cell], bhi = m.bbhi[cell];
  if (hi.x <= blo.x || lo.x >= bhi.x || hi.y <= blo.y || lo.y >= bhi.y || hi.z <= blo.z ||
      lo.z >= bhi.z)
    return 0.0;
  // cutting planes: cuts[] holds cell-plane indices, or ~j for plane j of a
  // box cell (taken from its bounds)
  int cuts[kMaxCellPlanes];
  Pl p0{0, 0, 0, 0}, p1 = p0, p2 = p0, p3 = p0;
  int ncut = 0;
  const double bb[6] = {blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z};
  if (m.isbox[cell]) {
    uint32_t mask;
    if (box_cuts(bb, c, T, mask) < 0) return 0.0;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
      const int j = __builtin_ctz(mm);
      const Pl pn = box_plane(bb, j, c);
      p3 = sel(ncut == 3, pn, p3);
      p2 = sel(ncut == 2, pn, p2);
      p1 = sel(ncut == 1, pn, p1);
      p0 = sel(ncut == 0, pn, p0);
      cuts[ncut] = ~j;
      ++ncut;
    }
  } else {
    for (int q = m.cf_off[cell], q1 = m.cf_off[cell] + m.npl[cell]; q < q1; ++q) {
      double4 cp = m.cpl[q];
      v3 nn = xyz4(cp);
      double off = cp.w - dot(nn, c);
      double d1 = off - dot(nn, T.b), d2 = off - dot(nn, T.c), d3 = off - dot(nn, T.d);
      double dmx = dmax(dmax(off, d1), dmax(d2, d3));
      double dmn = dmin(dmin(off, d1), dmin(d2, d3));
      if (dmx <= 0.0) return 0.0;
      if (dmn < 0.0) {
        Pl pn = mkpl(nn, off);
        p3 = sel(ncut == 3, pn, p3);
        p2 = sel(ncut == 2, pn, p2);
        p1 = sel(ncut == 1, pn, p1);
        p0 = sel(ncut == 0, pn, p0);
        if (ncut < kMaxCellPlanes) cuts[ncut] = q;
        ++ncut;
      }
    }
  }
  const bool need_cover = p.check_stencil || cl >= 2;
  if (four && !p.check_stencil && cl == 1 && ncut == kRegPlanes) {
    // four cutting planes and the PLIC plane: that plane counts only where it
    // crosses the tet (wholly kept: four planes; wholly removed: no phase)
    ++npairs;
    const Pl pl = plic_plane_at(s, cell, c);
    const D4 dp = plane_dists(T, pl);
    if (dmax(dmax(dp.a, dp.b), dmax(dp.c, dp.d)) <= 0.0) return 0.0;
    if (dmin(dmin(dp.a, dp.b), dmin(dp.c, dp.d)) >= 0.0) {
      dists4(T, p0, p1, p2, p3, four->row);
    } else {
      dists5(T, p0, p1, p2, p3, pl, four->row);
      four->five = true;
    }
    four->w = 1.0;
    four->on = true;
    return 0.0;
  }
  if (!poly_ok && ((cl == 1 && ncut >= kRegPlanes) || (need_cover && ncut > kRegPlanes)))
    return NAN;  // needs the polytope: the caller comes back with poly_ok
  ++npairs;  // a (tet, cell) pair with overlapping interiors
  // with `four` given (and no stencil check), a pair of exactly four planes
  // is handed back for the caller to evaluate
  if (four && !p.check_stencil && cl >= 2 && ncut == kRegPlanes) {
    dists4(T, p0, p1, p2, p3, four->row);
    four->w = cl == 3 ? s.alpha[cell] : 1.0;
    four->on = true;
    return 0.0;
  }
  double vc =
      (need_cover && ncut <= kRegPlanes) ? vol6_planes(T, det, p0, p1, p2, p3, ncut) : -1.0;
  double vph = 0.0;
  if (cl == 1) {
    double4 pp = s.plane[cell];
    v3 nn = xyz4(pp);
    double off = pp.w - dot(nn, c);
    if (four && !p.check_stencil && ncut == kRegPlanes - 1) {
      dists4(T, p0, p1, p2, mkpl(nn, off), four->row);
      four->w = 1.0;
      four->on = true;
      return 0.0;
    }
    if (ncut < kRegPlanes) {
      Pl pn = mkpl(nn, off);
      p3 = sel(ncut == 3, pn, p3);
      p2 = sel(ncut == 2, pn, p2);
      p1 = sel(ncut == 1, pn, p1);
      p0 = sel(ncut == 0, pn, p0);
      vph = vol6_planes(T, det, p0, p1, p2, p3, ncut + 1);
    } else {
      P.init_tet(T.a, T.b, T.c, T.d);
      bool ok = true;
      for (int q = 0; q < ncut && ok; ++q) {
        const Pl pc = cut_plane(m, cuts[q < kMaxCellPlanes ? q : 0], bb, c);
        ok = P.clip(mk3(pc.x, pc.y, pc.z), pc.w);
      }
      if (ok && vc < 0.0 && p.check_stencil) vc = P.vol6();
      ok = ok && P.clip(nn, off);
      vph = ok ? P.vol6() : 0.0;
      if (!ok || ncut > kMaxCellPlanes) ++ncap;
    }
  }
  if (need_cover && vc < 0.0) {
    P.init_tet(T.a, T.b, T.c, T.d);
    bool ok = true;
    for (int q = 0; q < ncut && ok; ++q) {
      const Pl pc = cut_plane(m, cuts[q < kMaxCellPlanes ? q : 0], bb, c);
      ok = P.clip(mk3(pc.x, pc.y, pc.z), pc.w);
    }
    vc = ok ? P.vol6() : 0.0;
    if (!ok || ncut > kMaxCellPlanes) ++ncap;
  }
  if (cl == 2) vph = vc;
  else if (cl == 3) vph = s.alpha[cell] * vc;
  if (p.check_stencil) *vcell = vc;
  return vph;
}

// Serial form over the whole stencil (host builds): the signed phase volume
// of flux tet k of face f; with check_stencil, *deficit receives the signed
// volume of the tet that no stencil cell covers and *gross its unsigned
// volume.
VHD double flux_tet_phase(const DMesh &m, const DState &s, const DParams &p, double dt,
                          double sc, int f, int k, Poly &P, unsigned long long &ncap,
                          unsigned long long &npairs, double *deficit, double *gross) {
  *deficit = 0.0;
  *gross = 0.0;
  v3 c, t1, t2, t3;
  double det, sgn;
  if (!flux_tet(m, s, dt, sc, f, k, c, t1, t2, t3, det, sgn)) return 0.0;
  const Tet T{mk3(0, 0, 0), t1, t2, t3};
  v3 lo, hi;
  tet_bbox(c, t1, t2, t3, lo, hi);
  double acc = 0.0, cover = 0.0;
  for (int e = m.st_off[f]; e < m.st_off[f + 1]; ++e) {
    double vc;
    acc += pair_phase6(m, s, p, c, T, det, lo, hi, m.st[e], P, ncap, npairs, &vc);
    cover += vc;
  }
  if (p.check_stencil) {
    *deficit = sgn * (det - cover) / 6.0;
    *gross = det / 6.0;
  }
  return sgn * acc / 6.0;
}

}  // namespace vof
