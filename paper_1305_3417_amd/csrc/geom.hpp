// geom.hpp -- double-precision geometry for the flux path, usable on the GPU and
// on the host (for the self-test entry point).
//
// Volumes of convex pieces of tetrahedra are what the phase flux needs
// (eqs. 2.22-2.23): a flux polyhedron is a signed sum of tetrahedra with apex
// at the face centre, and every tetrahedron is intersected with the planes of
// a stencil cell and, in interface cells, the PLIC half-space.  Two tools:
//
//  * tet_kept_fraction: the fraction of a tetrahedron on the kept side of one
//    plane as a function of the four signed vertex distances alone (affine
//    invariance), with no division by near-equal height differences.
//  * Poly: a convex polytope whose vertices all have exactly three
//    neighbours (a simple polytope), clipped plane by plane.  Each clip adds
//    one vertex per cut edge and links the new vertices around the cap by
//    walking the faces through the removed vertices.  The volume is summed
//    over the faces, each walked once and fanned from its first vertex.
//    Closed half-spaces: vertices on the plane are kept, so exactly
//    coplanar cell faces, face edges and sweep vectors need no tolerance.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define VHD __host__ __device__ __forceinline__

namespace vof {

struct v3 {
  double x, y, z;
};
VHD v3 mk3(double x, double y, double z) { return v3{x, y, z}; }
VHD v3 operator+(v3 a, v3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
VHD v3 operator-(v3 a, v3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
VHD v3 operator*(double s, v3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
VHD double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
VHD v3 cross(v3 a, v3 b) {
  return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// six times the signed volume of the tetrahedron (0, a, b, c)
VHD double det3(v3 a, v3 b, v3 c) { return dot(a, cross(b, c)); }
VHD double dmin(double a, double b) { return a < b ? a : b; }
VHD double dmax(double a, double b) { return a > b ? a : b; }

// A tetrahedron as four named vertices and four signed distances.  Every
// case analysis below first orders the vertices so that the kept ones
// (distance >= 0) come first, with a five-comparator sorting network on
// values; all later indexing is then by constant position, so nothing is
// indexed at run time and everything stays in registers.
struct Tet {
  v3 a, b, c, d;
};
struct D4 {
  double a, b, c, d;
};

// Component-wise select.  (A conditional expression on aggregate lvalues is
// lowered to a select of addresses, which forces them into memory.)
VHD v3 sel(bool c, v3 a, v3 b) {
  return v3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

VHD void cswap_kept(double &dx, double &dy) {
  bool sw = !(dx >= 0.0) && (dy >= 0.0);
  double t = dx;
  dx = sw ? dy : dx;
  dy = sw ? t : dy;
}

// kept vertices first (order among kept / among removed is immaterial)
VHD void sort_kept(D4 &d) {
  cswap_kept(d.a, d.b);
  cswap_kept(d.c, d.d);
  cswap_kept(d.a, d.c);
  cswap_kept(d.b, d.d);
  cswap_kept(d.b, d.c);
}

VHD int kept_count(const D4 &d) {
  return (d.a >= 0.0) + (d.b >= 0.0) + (d.c >= 0.0) + (d.d >= 0.0);
}

// Fraction of a tetrahedron with signed vertex distances d lying in the
// closed half-space d >= 0.  With t_xy = d_x / (d_x - d_y) the position of the
// cut on edge x -> y (x kept, y removed):
//   one kept vertex a:          t_ab t_ac t_ad
//   three kept (d removed):     1 - prod_j d_d / (d_d - d_j)
//   two kept (a, b):            t_ac t_ad + t_ad t_bc (1 - t_ac) + t_bc t_bd (1 - t_ad)
// (the last is the prism a, b | ac, ad, bc, bd cut into three tetrahedra).
// Each case is one quotient over a common denominator of positive factors
// (d_x >= 0 > d_y); with A = a - c, B = a - d, C = b - c, D = b - d the two-kept
// case is (a^2 C D - a b c D - b^2 d A) / (A B C D), every term positive.  The
// case is chosen by selects, so every lane performs a single division.
VHD double tet_kept_fraction(D4 d) {
  const int kept = kept_count(d);
  if (kept == 4) return 1.0;
  if (kept == 0) return 0.0;
  sort_kept(d);
  const double a = d.a, b = d.b, c = d.c, e = d.d;
  // one kept vertex
  const double n1 = a * a * a, q1 = (a - b) * (a - c) * (a - e);
  // three kept: the removed corner at e
  const double n3 = -(e * e * e), q3 = (a - e) * (b - e) * (c - e);
  // two kept
  const double A = a - c, B = a - e, C = b - c, D = b - e;
  const double n2 = a * a * C * D - a * b * c * D - b * b * e * A, q2 = A * B * C * D;
  const double num = kept == 1 ? n1 : (kept == 2 ? n2 : n3);
  const double den = kept == 1 ? q1 : (kept == 2 ? q2 : q3);
  const double r = num / den;
  return kept == 3 ? 1.0 - r : r;
}
VHD double tet_kept_fraction(const double dd[4]) {
  return tet_kept_fraction(D4{dd[0], dd[1], dd[2], dd[3]});
}

// ---------------------------------------------------------------------------
// register-only clipping of a tetrahedron by a few planes
// ---------------------------------------------------------------------------
// The part of a tetrahedron T on the kept side (d >= 0) of one plane is one
// or three tetrahedra whose vertices are vertices of T or cut points xy on
// edges x -> y (x kept, y removed) at parameter t_xy = d_x / (d_x - d_y).
// With the vertices sorted kept-first the pieces are consecutive windows of
// four in one sequence:
//   kept 1 (a):     [a, ab, ac, ad]            ratio t_ab t_ac t_ad
//   kept 2 (a, b):  [a, ac, ad, b, bc, bd]     ratios t_ac t_ad, t_ad t_bc (1 - t_ac),
//                                                      t_bc t_bd (1 - t_ad)
//   kept 3 (a,b,c): [a, b, c, ad, bd, cd]      ratios t_ad, (1 - t_ad) t_bd,
//                                                      (1 - t_ad)(1 - t_bd) t_cd
//   kept 4:         [a, b, c, d]               ratio 1
// where the ratio of a piece is its volume over |T| (the determinant of the
// barycentric coordinates of its vertices).  A cut point's signed distances
// to the other planes interpolate those of its edge's ends, so clipping by
// several planes needs only the 4 x K matrix of vertex distances: |T ∩ H_0
// ∩ ... ∩ H_K-1| = |T| * sum over pieces of ratio * (fraction of the piece
// kept by the remaining planes).

// signed distances of one vertex to the K planes still to apply
template <int K>
struct VD {
  double d[K];
};
template <int K>
struct TD {
  VD<K> a, b, c, e;
};

template <int K>
VHD VD<K> sel(bool c, const VD<K> &x, const VD<K> &y) {
  VD<K> r;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = c ? x.d[k] : y.d[k];
  return r;
}

// distances to planes 1..K-1 of the cut point on edge x -> y
template <int K>
VHD VD<K - 1> cut_rest(const VD<K> &x, const VD<K> &y, double t) {
  VD<K - 1> r;
#pragma unroll
  for (int k = 1; k < K; ++k) r.d[k - 1] = x.d[k] + t * (y.d[k] - x.d[k]);
  return r;
}
template <int K>
VHD VD<K - 1> rest(const VD<K> &x) {
  VD<K - 1> r;
#pragma unroll
  for (int k = 1; k < K; ++k) r.d[k - 1] = x.d[k];
  return r;
}

template <int K>
VHD void cswap_kept(VD<K> &x, VD<K> &y) {
  bool sw = !(x.d[0] >= 0.0) && (y.d[0] >= 0.0);
  VD<K> t = x;
  x = sel(sw, y, x);
  y = sel(sw, t, y);
}

// edge parameter of the cut on x -> y for plane 0 (x kept, y removed; 0
// when unused)
template <int K>
VHD double tcut(const VD<K> &x, const VD<K> &y) {
  double den = x.d[0] - y.d[0];
  return den > 0.0 ? x.d[0] / den : 0.0;
}

// fraction of a tetrahedron kept by all K planes, from its vertex distances
template <int K>
VHD double kept_fraction(TD<K> T);

template <>
VHD double kept_fraction<1>(TD<1> T) {
  return tet_kept_fraction(D4{T.a.d[0], T.b.d[0], T.c.d[0], T.e.d[0]});
}

// The kept part of a tetrahedron under its first plane as at most three
// tetrahedra: piece i is the window S_i..S_i+3 of a six-point sequence of
// vertices and cut points, carrying the distances to the other planes, with
// volume ratio r_i to the whole; n pieces (0 when nothing is kept).
template <int K>
struct Split {
  VD<K - 1> S0, S1, S2, S3, S4, S5;
  double r0, r1, r2;
  int n;
};

template <int K>
VHD Split<K> split_first(TD<K> T) {
  const int kept = (T.a.d[0] >= 0.0) + (T.b.d[0] >= 0.0) + (T.c.d[0] >= 0.0) +
                   (T.e.d[0] >= 0.0);
  cswap_kept(T.a, T.b);
  cswap_kept(T.c, T.e);
  cswap_kept(T.a, T.c);
  cswap_kept(T.b, T.e);
  cswap_kept(T.b, T.c);
  const bool k1 = kept == 1, k2 = kept == 2, k3 = kept == 3, k4 = kept == 4;
  // the four cut points any case needs: A = ad, B = ab | ac, C = ac | bc | bd,
  // D = bd | cd (for kept 1 | 2 | 3)
  const double tA = tcut(T.a, T.e);
  const VD<K> Bto = sel(k1, T.b, T.c);
  const double tB = tcut(T.a, Bto);
  const VD<K> Cfrom = sel(k1, T.a, T.b);
  const VD<K> Cto = sel(k3, T.e, T.c);
  const double tC = tcut(Cfrom, Cto);
  const VD<K> Dfrom = sel(k3, T.c, T.b);
  const double tD = tcut(Dfrom, T.e);
  const VD<K - 1> A = cut_rest(T.a, T.e, tA);
  const VD<K - 1> B = cut_rest(T.a, Bto, tB);
  const VD<K - 1> C = cut_rest(Cfrom, Cto, tC);
  const VD<K - 1> D = cut_rest(Dfrom, T.e, tD);
  const VD<K - 1> ra = rest(T.a), rb = rest(T.b), rc = rest(T.c), re = rest(T.e);
  Split<K> sp;
  // the sequence of piece vertices
  sp.S0 = ra;
  sp.S1 = sel(k3 || k4, rb, B);
  sp.S2 = sel(k1, C, sel(k2, A, rc));
  sp.S3 = sel(k2, rb, sel(k4, re, A));
  sp.S4 = C;
  sp.S5 = D;
  sp.r0 = k4 ? 1.0 : (k1 ? tB * tC * tA : (k2 ? tB * tA : tA));
  sp.r1 = k2 ? tA * tC * (1.0 - tB) : (1.0 - tA) * tC;
  sp.r2 = k2 ? tC * tD * (1.0 - tA) : (1.0 - tA) * (1.0 - tC) * tD;
  sp.n = kept == 0 ? 0 : ((k1 || k4) ? 1 : 3);
  return sp;
}

// piece i of a split and its volume ratio
template <int K>
VHD TD<K - 1> split_piece(const Split<K> sp, int i, double &r) {
  r = i == 0 ? sp.r0 : (i == 1 ? sp.r1 : sp.r2);
  return TD<K - 1>{sel(i == 0, sp.S0, sel(i == 1, sp.S1, sp.S2)),
                   sel(i == 0, sp.S1, sel(i == 1, sp.S2, sp.S3)),
                   sel(i == 0, sp.S2, sel(i == 1, sp.S3, sp.S4)),
                   sel(i == 0, sp.S3, sel(i == 1, sp.S4, sp.S5))};
}

// The pieces are written out one by one (the same sums in the same order as
// a loop over split_piece), so that each piece's window of the sequence is
// fixed at compile time rather than chosen by selects.
template <int K>
VHD double kept_fraction(TD<K> T) {
  const Split<K> sp = split_first<K>(T);
  double acc = 0.0;
  if (sp.n >= 1) acc += sp.r0 * kept_fraction<K - 1>(TD<K - 1>{sp.S0, sp.S1, sp.S2, sp.S3});
  if (sp.n >= 2) {
    acc += sp.r1 * kept_fraction<K - 1>(TD<K - 1>{sp.S1, sp.S2, sp.S3, sp.S4});
    acc += sp.r2 * kept_fraction<K - 1>(TD<K - 1>{sp.S2, sp.S3, sp.S4, sp.S5});
  }
  return acc;
}

// A plane n.x = s as four plain doubles (plain aggregates stay in registers
// through selects, unlike the union-based vector types).
struct Pl {
  double x, y, z, w;
};
VHD Pl mkpl(v3 n, double s) { return Pl{n.x, n.y, n.z, s}; }
VHD Pl sel(bool c, Pl a, Pl b) {
  return Pl{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w};
}

// distances s - n.x of the four vertices to the plane (n, s)
VHD D4 plane_dists(const Tet &t, Pl pl) {
  v3 n = mk3(pl.x, pl.y, pl.z);
  return D4{pl.w - dot(n, t.a), pl.w - dot(n, t.b), pl.w - dot(n, t.c), pl.w - dot(n, t.d)};
}

// Number of planes a (tetrahedron, cell) pair may have on the register path.
constexpr int kRegPlanes = 4;

// six times |T ∩ {n_j.x <= s_j, j < k}| for k <= KMAX <= kRegPlanes planes,
// T positively ordered with six times its volume vol6
template <int KMAX = kRegPlanes>
VHD double vol6_planes(const Tet &T, double vol6, Pl p0, Pl p1, Pl p2, Pl p3, int k) {
  static_assert(KMAX >= 1 && KMAX <= kRegPlanes, "plane count");
  if (k == 0) return vol6;
  const D4 d0 = plane_dists(T, p0);
  if (KMAX == 1 || k == 1) return vol6 * tet_kept_fraction(d0);
  const D4 d1 = plane_dists(T, p1);
  if (KMAX == 2 || k == 2)
    return vol6 * kept_fraction<2>(TD<2>{{{d0.a, d1.a}}, {{d0.b, d1.b}}, {{d0.c, d1.c}},
                                         {{d0.d, d1.d}}});
  const D4 d2 = plane_dists(T, p2);
  if constexpr (KMAX == 3) {
    return vol6 * kept_fraction<3>(TD<3>{{{d0.a, d1.a, d2.a}}, {{d0.b, d1.b, d2.b}},
                                         {{d0.c, d1.c, d2.c}}, {{d0.d, d1.d, d2.d}}});
  } else {
    if (k == 3)
      return vol6 * kept_fraction<3>(TD<3>{{{d0.a, d1.a, d2.a}}, {{d0.b, d1.b, d2.b}},
                                           {{d0.c, d1.c, d2.c}}, {{d0.d, d1.d, d2.d}}});
    const D4 d3 = plane_dists(T, p3);
    return vol6 * kept_fraction<4>(TD<4>{{{d0.a, d1.a, d2.a, d3.a}},
                                         {{d0.b, d1.b, d2.b, d3.b}},
                                         {{d0.c, d1.c, d2.c, d3.c}},
                                         {{d0.d, d1.d, d2.d, d3.d}}});
  }
}

// distances of the tet's vertices to the first K of five planes (vertex by
// vertex)
template <int K>
VHD TD<K> dist_table(const Tet &T, Pl p0, Pl p1, Pl p2, Pl p3, Pl p4 = Pl{0, 0, 0, 0}) {
  const Pl pl[5] = {p0, p1, p2, p3, p4};
  TD<K> D;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const D4 d = plane_dists(T, pl[k]);
    D.a.d[k] = d.a;
    D.b.d[k] = d.b;
    D.c.d[k] = d.c;
    D.e.d[k] = d.d;
  }
  return D;
}

// Term i of kept_fraction<K>(D): piece i of the first plane's split, its
// volume ratio times the fraction of it the other planes keep (0 past the
// split's pieces).  kept_fraction<K> adds the terms for i = 0, 1, 2 in order.
template <int K>
VHD double split_term(const TD<K> &D, int i) {
  const Split<K> sp = split_first<K>(D);
  if (i >= sp.n) return 0.0;
  double r;
  const TD<K - 1> pc = split_piece<K>(sp, i, r);
  return r * kept_fraction<K - 1>(pc);
}

// Term (i, j) two levels down: piece i of the first plane's split (its ratio
// in *ri, 0 past the split's pieces) and term j of that piece's own split.
// kept_fraction<K>(D) is the sum over i of r_i times the sum over j.
template <int K>
VHD double split_term2(const TD<K> &D, int i, int j, double &ri) {
  const Split<K> sp = split_first<K>(D);
  ri = 0.0;
  if (i >= sp.n) return 0.0;
  const TD<K - 1> pc = split_piece<K>(sp, i, ri);
  return split_term<K - 1>(pc, j);
}

// ---------------------------------------------------------------------------
// simple polytope as a vertex graph
// ---------------------------------------------------------------------------
// Vertex i has position (X, Y, Z) and neighbours NB(i,0..2) in counter-clockwise
// order seen from outside.  Face F(i,k) is the wedge between edges i->NB(i,k)
// and i->NB(i,k+1); walked counter-clockwise it passes NB(i,k+1) -> i -> NB(i,k).
// Arriving at vertex v from u, the next vertex of the same face is
// NB(v, (index of u in v) + 2 mod 3).
//
// Storage is strided so that a wavefront can keep one polytope per lane in
// LDS with consecutive lanes in consecutive words.
struct Poly {
  double *px, *py, *pz, *ps;  // position and signed distance, element i at [i * st]
  uint8_t *nb;                // neighbour (i, k) at [(3 i + k) * st]
  uint8_t *aux;               // scratch byte per vertex at [i * st]
  int st;                     // element stride
  int nv;                     // vertex count
  int cap;                    // vertex capacity

  VHD double &X(int i) { return px[i * st]; }
  VHD double &Y(int i) { return py[i * st]; }
  VHD double &Z(int i) { return pz[i * st]; }
  VHD double &SD(int i) { return ps[i * st]; }
  VHD uint8_t &NB(int i, int k) { return nb[(3 * i + k) * st]; }
  VHD uint8_t &AUX(int i) { return aux[i * st]; }
  VHD v3 P(int i) { return mk3(X(i), Y(i), Z(i)); }
  VHD void setP(int i, v3 p) { X(i) = p.x; Y(i) = p.y; Z(i) = p.z; }
  VHD int slot(int v, int u) {  // index of neighbour u in vertex v
    return NB(v, 0) == u ? 0 : (NB(v, 1) == u ? 1 : 2);
  }

  // positively oriented tetrahedron (a, b, c, d): det(b - a, c - a, d - a) > 0
  VHD void init_tet(v3 a, v3 b, v3 c, v3 d) {
    nv = 4;
    setP(0, a); setP(1, b); setP(2, c); setP(3, d);
    NB(0, 0) = 1; NB(0, 1) = 3; NB(0, 2) = 2;
    NB(1, 0) = 0; NB(1, 1) = 2; NB(1, 2) = 3;
    NB(2, 0) = 0; NB(2, 1) = 3; NB(2, 2) = 1;
    NB(3, 0) = 0; NB(3, 1) = 1; NB(3, 2) = 2;
  }

  // Keep {x : n.x <= s}.  Returns false on capacity overflow or an
  // inconsistent cap (the polytope must then be discarded by the caller).
  VHD bool clip(v3 n, double s) {
    if (nv == 0) return true;
    // A vertex within 1e-13 of the polytope's extent of the plane lies on it
    // (kept): rounding noise on vertices that are on the plane cannot then
    // cut a sliver of zero width off the polytope.
    double ext = 0.0;
    for (int i = 1; i < nv; ++i)
      ext = dmax(ext, dmax(fabs(X(i) - X(0)), dmax(fabs(Y(i) - Y(0)), fabs(Z(i) - Z(0)))));
    const double tol = 1e-13 * sqrt(dot(n, n)) * ext;
    bool anyneg = false, anypos = false;
    for (int i = 0; i < nv; ++i) {
      double d = s - (n.x * X(i) + n.y * Y(i) + n.z * Z(i));
      if (fabs(d) <= tol) d = 0.0;
      SD(i) = d;
      anyneg |= d < 0.0;
      anypos |= d > 0.0;
    }
    if (!anyneg) return true;
    if (!anypos) { nv = 0; return true; }
    const int onv = nv;
    int m = nv;
    // one new vertex on every edge from a kept to a removed vertex
    for (int u = 0; u < onv; ++u) {
      double du = SD(u);
      if (du < 0.0) continue;
      for (int k = 0; k < 3; ++k) {
        int v = NB(u, k);
        if (v >= onv) continue;
        double dv = SD(v);
        if (dv >= 0.0) continue;
        if (m >= cap) return false;
        double t = du / (du - dv);
        setP(m, mk3(X(u) + t * (X(v) - X(u)), Y(u) + t * (Y(v) - Y(u)),
                    Z(u) + t * (Z(v) - Z(u))));
        NB(m, 0) = (uint8_t)u;
        NB(m, 1) = 255;
        NB(m, 2) = 255;
        AUX(m) = (uint8_t)v;  // removed end of the cut edge
        NB(u, k) = (uint8_t)m;
        ++m;
      }
    }
    // link the cap: from the kept end u of a new vertex w, walk the face that
    // contains u -> (removed end) through removed vertices until a kept
    // vertex is reached; the new vertex on that exit edge follows w on the cap
    for (int w = onv; w < m; ++w) {
      int prev = NB(w, 0), cur = AUX(w);
      for (int guard = 0; guard < 3 * onv; ++guard) {
        int nx = NB(cur, (slot(cur, prev) + 2) % 3);
        prev = cur;
        cur = nx;
        if (SD(cur) >= 0.0) break;
      }
      int w2 = -1;
      if (SD(cur) >= 0.0)
        for (int k = 0; k < 3; ++k) {
          int c = NB(cur, k);
          if (c >= onv && c < m && AUX(c) == prev) w2 = c;
        }
      if (w2 < 0) { nv = 0; return false; }  // inconsistent cap: report, never index out
      NB(w, 2) = (uint8_t)w2;
      NB(w2, 1) = (uint8_t)w;
    }
    // every cap vertex needs two distinct cap neighbours; anything else is a
    // graph that rounding has made inconsistent: report it, never index out
    for (int w = onv; w < m; ++w) {
      const int a = NB(w, 1), b = NB(w, 2);
      if (a < onv || a >= m || b < onv || b >= m || a == b) { nv = 0; return false; }
    }
    // compact: kept originals and new vertices, in order
    int q = 0;
    for (int i = 0; i < m; ++i) {
      bool keep = (i >= onv) || (SD(i) >= 0.0);
      AUX(i) = keep ? (uint8_t)(q++) : (uint8_t)255;
    }
    for (int i = 0; i < m; ++i) {
      int j = AUX(i);
      if (j == 255 || j == i) continue;
      X(j) = X(i); Y(j) = Y(i); Z(j) = Z(i);
      NB(j, 0) = NB(i, 0); NB(j, 1) = NB(i, 1); NB(j, 2) = NB(i, 2);
    }
    for (int j = 0; j < q; ++j)
      for (int k = 0; k < 3; ++k) NB(j, k) = AUX(NB(j, k));
    nv = q;
    return true;
  }

  // six times the volume: every face walked once, fanned from its first vertex
  VHD double vol6() {
    if (nv == 0) return 0.0;
    for (int i = 0; i < nv; ++i) AUX(i) = 0;
    v3 o = P(0);
    double v = 0.0;
    for (int u = 0; u < nv; ++u) {
      for (int k = 0; k < 3; ++k) {
        if (AUX(u) & (1 << k)) continue;
        AUX(u) |= (uint8_t)(1 << k);
        v3 a = P(u) - o;
        int prev = u, cur = NB(u, k);
        v3 b = P(cur) - o;
        for (int guard = 0; guard < 3 * nv && cur != u; ++guard) {
          int kn = (slot(cur, prev) + 2) % 3;
          AUX(cur) |= (uint8_t)(1 << kn);
          int nx = NB(cur, kn);
          if (nx != u) {
            v3 c = P(nx) - o;
            v += det3(a, b, c);
            b = c;
          }
          prev = cur;
          cur = nx;
        }
      }
    }
    return v;
  }
};

}  // namespace vof
