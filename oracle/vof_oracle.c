/*
 * vof_oracle.c -- plain, slow, CPU reference of the geometric PLIC VoF flux path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU
 * library is checked.  It is called from the tests, from the package's smoke
 * check and from the benchmark's CPU-baseline leg; the product path never
 * loads it.  It shares no code, header or table with the GPU library.
 *
 * Everything is double precision.  Each function names the passage of
 * Maric, Marschall & Bothe, "voFoam - A geometrical Volume of Fluid algorithm
 * on arbitrary unstructured meshes ..." (arXiv:1305.3417) that it follows.
 * Where the paper is silent the reading used is stated in a comment marked
 * READING.  The algorithms follow the paper's steps in its order:
 *
 *   geometry          Section 2 (face centre = mean of points, area vectors,
 *                     owner/neighbour orientation, eqs. 2.4-2.5)
 *   point velocity    inverse-distance weighting, eqs. 2.6-2.7, applied to U
 *   flux polyhedron   swept face along point trajectories (eq. 2.16), volume by
 *                     tetrahedral decomposition (eqs. 2.18-2.19)
 *   flux correction   secant iteration on the sweep length until the volume
 *                     equals |F_f| dt (eq. 2.17), no topology change
 *   reconstruction    Algorithm 1: NAG gradient (eqs. 2.6-2.12), then
 *                     secant / bisection positioning (Section 2.2.2)
 *   phase flux        S_f clipped by each stencil cell (eq. 2.22), then by
 *                     the PLIC half-space in interface cells (eq. 2.23), by
 *                     plane clipping and capping (Section 2.1)
 *   update            eq. 2.2 with owner/neighbour signs (eq. 2.5); optionally
 *                     only outside the bulk (the narrow band, Section 2.3)
 *   wisps             optional conservative redistribution of wisps to the
 *                     interface cells around them (Section 2.3)
 *   mapping           volume fraction on a changed mesh from the old
 *                     reconstruction (Section 3, Algorithm 2)
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so vof_oracle.c -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_MAXV 96   /* vertices of one clipped polyhedron            */
#define O_MAXF 48   /* faces of one clipped polyhedron               */
#define O_MAXFV 48  /* vertices of one face                          */
#define O_MAXN 16   /* points of one mesh face                       */

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static void v_sub(const double *a, const double *b, double *r) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void v_cross(const double *a, const double *b, double *r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_dot(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double v_norm(const double *a) { return sqrt(v_dot(a, a)); }
/* det(a - o, b - o, c - o) = six times the signed tet volume (o, a, b, c) */
static double tet6(const double *o, const double *a, const double *b, const double *c) {
  double u[3], v[3], w[3], x[3];
  v_sub(a, o, u); v_sub(b, o, v); v_sub(c, o, w);
  v_cross(v, w, x);
  return v_dot(u, x);
}

/* ------------------------------------------------------------------ */
/* convex polyhedron with outward counter-clockwise faces (Section 2.1) */
/* ------------------------------------------------------------------ */
typedef struct {
  int nv, nf;
  double v[O_MAXV][3];
  int fn[O_MAXF];
  int fv[O_MAXF][O_MAXFV];
} opoly;

/* Volume by the divergence theorem: fan triangles of every face against a
 * reference point. */
static double opoly_volume(const opoly *P) {
  if (P->nv == 0 || P->nf == 0) return 0.0;
  const double *r = P->v[0];
  double vol = 0.0;
  for (int f = 0; f < P->nf; ++f) {
    const int *L = P->fv[f];
    for (int k = 1; k + 1 < P->fn[f]; ++k)
      vol += tet6(r, P->v[L[0]], P->v[L[k]], P->v[L[k + 1]]);
  }
  return vol / 6.0;
}

/* Plane clipping and capping (Section 2.1, the modified Ahn-Shashkov
 * algorithm): every face is clipped against the half-space {x : n.x <= s};
 * points created on cut edges are shared between the two faces of the edge
 * (no repeated points); the cap face is then formed from the cut points and
 * the kept vertices on the plane, ordered by an insertion sort of their angle
 * about the cap centre.  Half-spaces are closed: vertices on the plane are
 * kept.  A clipped face whose vertices are all cap points lies in the plane
 * (or has no area) and is replaced by the cap, so a face that rounding
 * leaves a hair outside the plane is not counted twice.
 * Returns 0 on success, -1 on capacity overflow. */
static int opoly_clip(opoly *P, const double *n, double s) {
  if (P->nv == 0) return 0;
  double d[O_MAXV];
  int any_in = 0, any_out = 0;
  /* READING: the paper's clip-and-cap treats the void / point / edge / face /
   * whole special cases internally (Section 2.1).  Here a vertex whose
   * distance to the plane is below 1e-13 of the polytope's extent counts as
   * on the plane, so rounding cannot split a face lying in the plane. */
  double ext = 0.0;
  for (int i = 1; i < P->nv; ++i)
    for (int c = 0; c < 3; ++c) ext = fmax(ext, fabs(P->v[i][c] - P->v[0][c]));
  double tol = 1e-13 * v_norm(n) * ext;
  for (int i = 0; i < P->nv; ++i) {
    d[i] = v_dot(n, P->v[i]) - s;
    if (fabs(d[i]) <= tol) d[i] = 0.0;
    if (d[i] < 0.0) any_in = 1;
    if (d[i] > 0.0) any_out = 1;
  }
  if (!any_out) return 0;                 /* whole polyhedron kept    */
  if (!any_in) { P->nv = 0; P->nf = 0; return 0; }  /* void or degenerate */

  opoly Q;
  Q.nv = 0; Q.nf = 0;
  int map[O_MAXV];
  for (int i = 0; i < P->nv; ++i) map[i] = -1;
  /* cut-edge cache: (a, b) unordered -> new vertex */
  int ea[O_MAXV * 3], eb[O_MAXV * 3], ev[O_MAXV * 3], ne = 0;
  int cap[O_MAXV], ncap = 0;

  for (int f = 0; f < P->nf; ++f) {
    int out[O_MAXFV], no = 0;
    int m = P->fn[f];
    for (int k = 0; k < m; ++k) {
      int a = P->fv[f][k], b = P->fv[f][(k + 1) % m];
      if (d[a] <= 0.0) {
        if (map[a] < 0) {
          if (Q.nv >= O_MAXV) return -1;
          map[a] = Q.nv;
          memcpy(Q.v[Q.nv], P->v[a], sizeof(double) * 3);
          ++Q.nv;
          if (d[a] == 0.0) cap[ncap++] = map[a];
        }
        if (no >= O_MAXFV) return -1;
        out[no++] = map[a];
      }
      if ((d[a] < 0.0 && d[b] > 0.0) || (d[a] > 0.0 && d[b] < 0.0)) {
        int lo = a < b ? a : b, hi = a < b ? b : a, idx = -1;
        for (int e = 0; e < ne; ++e)
          if (ea[e] == lo && eb[e] == hi) { idx = ev[e]; break; }
        if (idx < 0) {
          if (Q.nv >= O_MAXV) return -1;
          /* interpolate from the kept end towards the removed end */
          int pin = d[a] < 0.0 ? a : b, pout = d[a] < 0.0 ? b : a;
          double t = d[pin] / (d[pin] - d[pout]);
          for (int c = 0; c < 3; ++c)
            Q.v[Q.nv][c] = P->v[pin][c] + t * (P->v[pout][c] - P->v[pin][c]);
          idx = Q.nv++;
          ea[ne] = lo; eb[ne] = hi; ev[ne] = idx; ++ne;
          cap[ncap++] = idx;
        }
        if (no >= O_MAXFV) return -1;
        out[no++] = idx;
      }
    }
    if (no >= 3) {
      if (Q.nf >= O_MAXF) return -1;
      Q.fn[Q.nf] = no;
      memcpy(Q.fv[Q.nf], out, sizeof(int) * no);
      ++Q.nf;
    }
  }

  /* faces made only of cap points lie in the plane: the cap replaces them */
  {
    int oncap[O_MAXV];
    for (int i = 0; i < Q.nv; ++i) oncap[i] = 0;
    for (int i = 0; i < ncap; ++i) oncap[cap[i]] = 1;
    int kept = 0;
    for (int f = 0; f < Q.nf; ++f) {
      int all = 1;
      for (int k = 0; k < Q.fn[f]; ++k) all &= oncap[Q.fv[f][k]];
      if (all) continue;
      if (kept != f) {
        Q.fn[kept] = Q.fn[f];
        memcpy(Q.fv[kept], Q.fv[f], sizeof(int) * Q.fn[f]);
      }
      ++kept;
    }
    Q.nf = kept;
  }
  if (ncap >= 3) {
    /* cap centre and an in-plane basis (u, w) with u x w along n */
    double c[3] = {0, 0, 0};
    for (int i = 0; i < ncap; ++i)
      for (int k = 0; k < 3; ++k) c[k] += Q.v[cap[i]][k];
    for (int k = 0; k < 3; ++k) c[k] /= ncap;
    double u[3] = {0, 0, 0}, w[3];
    double far = -1.0;
    for (int i = 0; i < ncap; ++i) {
      double r[3];
      v_sub(Q.v[cap[i]], c, r);
      double l = v_norm(r);
      if (l > far) { far = l; memcpy(u, r, sizeof u); }
    }
    if (far > 0.0) {
      /* remove the normal part of u, then normalise */
      double nn = v_dot(n, n), un = v_dot(u, n) / nn;
      for (int k = 0; k < 3; ++k) u[k] -= un * n[k];
      double lu = v_norm(u);
      for (int k = 0; k < 3; ++k) u[k] /= lu;
      v_cross(n, u, w);
      double lw = v_norm(w);
      for (int k = 0; k < 3; ++k) w[k] /= lw;
      double ang[O_MAXV];
      for (int i = 0; i < ncap; ++i) {
        double r[3];
        v_sub(Q.v[cap[i]], c, r);
        ang[i] = atan2(v_dot(r, w), v_dot(r, u));
      }
      /* insertion sort by angle: counter-clockwise about +n, i.e. the cap's
       * outward normal points into the removed half-space */
      for (int i = 1; i < ncap; ++i) {
        double a = ang[i]; int id = cap[i]; int j = i - 1;
        while (j >= 0 && ang[j] > a) { ang[j + 1] = ang[j]; cap[j + 1] = cap[j]; --j; }
        ang[j + 1] = a; cap[j + 1] = id;
      }
      if (Q.nf >= O_MAXF || ncap > O_MAXFV) return -1;
      Q.fn[Q.nf] = ncap;
      memcpy(Q.fv[Q.nf], cap, sizeof(int) * ncap);
      ++Q.nf;
    }
  }
  *P = Q;
  return 0;
}

static void opoly_tet(opoly *P, const double *a, const double *b, const double *c,
                      const double *d) {
  /* positively oriented tet (a, b, c, d): outward faces (b,c,d) (a,d,c) (a,b,d) (a,c,b) */
  P->nv = 4; P->nf = 4;
  memcpy(P->v[0], a, 24); memcpy(P->v[1], b, 24);
  memcpy(P->v[2], c, 24); memcpy(P->v[3], d, 24);
  static const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  for (int f = 0; f < 4; ++f) {
    P->fn[f] = 3;
    for (int k = 0; k < 3; ++k) P->fv[f][k] = F[f][k];
  }
}

/* ------------------------------------------------------------------ */
/* mesh, derived addressing and geometry (Section 2)                   */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t np, nc, nf, ni;
  double *x;                 /* 3 np                                   */
  int64_t *foff;             /* nf + 1                                 */
  int32_t *fpts;
  int32_t *own, *nei;        /* nf, ni                                 */
  int64_t *cf_off;           /* cell -> faces                          */
  int32_t *cf_face;
  int8_t *cf_sign;           /* +1 owner, -1 neighbour (eq. 2.5)       */
  int64_t *pc_off;           /* point -> cells (sorted)                */
  int32_t *pc_cell;
  double *w_pc;              /* IDW weights (eq. 2.7)                  */
  int64_t *st_off;           /* face stencil: cells of the face points */
  int32_t *st_cell;
  double *V, *xc;            /* cell volume, centroid                  */
  double *S, *cfc;           /* face area vector, face centre          */
  double *Up;                /* point velocity (3 np)                  */
  double *F0;                /* reference face flux                    */
  /* last reconstruction */
  int8_t *cls;               /* 0 empty, 1 interface, 2 full, 3 fallback */
  double *pn;                /* plane normal (3 nc)                    */
  double *ps;                /* plane position                         */
  double *grad;              /* NAG gradient (3 nc)                    */
  double eps;                /* reconstruction tolerance               */
  int grad_kind;             /* 0 NAG (Section 2.2.1), 1 generalized LSQ */
  int band;                  /* 1: bulk cells are not updated (Section 2.3) */
  int wisps;                 /* 1: wisps redistributed after the update */
} omesh;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Mean of the face points: the face centre of Section 2.2.1. */
static void face_centre(const omesh *M, int64_t f, double *c) {
  int64_t b = M->foff[f], e = M->foff[f + 1];
  c[0] = c[1] = c[2] = 0.0;
  for (int64_t k = b; k < e; ++k)
    for (int j = 0; j < 3; ++j) c[j] += M->x[3 * (int64_t)M->fpts[k] + j];
  for (int j = 0; j < 3; ++j) c[j] /= (double)(e - b);
}

/* Cell c as a polyhedron with outward faces (owner faces as stored,
 * neighbour faces reversed). */
static int cell_poly(const omesh *M, int64_t c, opoly *P) {
  int gl[O_MAXV], ng = 0;
  P->nv = 0; P->nf = 0;
  for (int64_t k = M->cf_off[c]; k < M->cf_off[c + 1]; ++k) {
    int64_t f = M->cf_face[k];
    int sg = M->cf_sign[k];
    int64_t b = M->foff[f], n = M->foff[f + 1] - b;
    if (P->nf >= O_MAXF || n > O_MAXFV) return -1;
    for (int64_t i = 0; i < n; ++i) {
      int p = M->fpts[b + (sg > 0 ? i : (n - 1 - i))];
      int idx = -1;
      for (int j = 0; j < ng; ++j) if (gl[j] == p) { idx = j; break; }
      if (idx < 0) {
        if (ng >= O_MAXV) return -1;
        gl[ng] = p; idx = ng++;
        memcpy(P->v[idx], &M->x[3 * (int64_t)p], 24);
      }
      P->fv[P->nf][i] = idx;
    }
    P->fn[P->nf++] = (int)n;
  }
  P->nv = ng;
  return 0;
}

omesh *orc_create(int64_t np, int64_t nc, int64_t nf, int64_t ni, const double *pts,
                  const int64_t *foff, const int32_t *fpts, const int32_t *own,
                  const int32_t *nei) {
  omesh *M = (omesh *)calloc(1, sizeof(omesh));
  M->np = np; M->nc = nc; M->nf = nf; M->ni = ni;
  M->eps = 1e-12;
  int64_t nfp = foff[nf];
  M->x = malloc(sizeof(double) * 3 * np); memcpy(M->x, pts, sizeof(double) * 3 * np);
  M->foff = malloc(sizeof(int64_t) * (nf + 1)); memcpy(M->foff, foff, sizeof(int64_t) * (nf + 1));
  M->fpts = malloc(sizeof(int32_t) * nfp); memcpy(M->fpts, fpts, sizeof(int32_t) * nfp);
  M->own = malloc(sizeof(int32_t) * nf); memcpy(M->own, own, sizeof(int32_t) * nf);
  M->nei = malloc(sizeof(int32_t) * (ni > 0 ? ni : 1));
  if (ni) memcpy(M->nei, nei, sizeof(int32_t) * ni);

  /* cell -> faces with owner / neighbour sign (eq. 2.5) */
  M->cf_off = calloc(nc + 1, sizeof(int64_t));
  for (int64_t f = 0; f < nf; ++f) {
    M->cf_off[own[f] + 1]++;
    if (f < ni) M->cf_off[nei[f] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) M->cf_off[c + 1] += M->cf_off[c];
  M->cf_face = malloc(sizeof(int32_t) * M->cf_off[nc]);
  M->cf_sign = malloc(M->cf_off[nc]);
  int64_t *fill = calloc(nc, sizeof(int64_t));
  for (int64_t f = 0; f < nf; ++f) {
    int64_t c = own[f];
    M->cf_face[M->cf_off[c] + fill[c]] = (int32_t)f; M->cf_sign[M->cf_off[c] + fill[c]] = 1; fill[c]++;
    if (f < ni) {
      c = nei[f];
      M->cf_face[M->cf_off[c] + fill[c]] = (int32_t)f; M->cf_sign[M->cf_off[c] + fill[c]] = -1; fill[c]++;
    }
  }
  free(fill);

  /* point -> cells: every cell that has a face containing the point */
  int64_t *cnt = calloc(np + 1, sizeof(int64_t));
  for (int64_t f = 0; f < nf; ++f)
    for (int64_t k = foff[f]; k < foff[f + 1]; ++k) cnt[fpts[k] + 1] += (f < ni) ? 2 : 1;
  for (int64_t p = 0; p < np; ++p) cnt[p + 1] += cnt[p];
  int32_t *tmp = malloc(sizeof(int32_t) * (cnt[np] > 0 ? cnt[np] : 1));
  int64_t *tf = calloc(np, sizeof(int64_t));
  for (int64_t f = 0; f < nf; ++f)
    for (int64_t k = foff[f]; k < foff[f + 1]; ++k) {
      int64_t p = fpts[k];
      tmp[cnt[p] + tf[p]++] = own[f];
      if (f < ni) tmp[cnt[p] + tf[p]++] = nei[f];
    }
  M->pc_off = calloc(np + 1, sizeof(int64_t));
  for (int64_t p = 0; p < np; ++p) {
    qsort(tmp + cnt[p], tf[p], sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t k = 0; k < tf[p]; ++k)
      if (k == 0 || tmp[cnt[p] + k] != tmp[cnt[p] + k - 1]) ++u;
    M->pc_off[p + 1] = M->pc_off[p] + u;
  }
  M->pc_cell = malloc(sizeof(int32_t) * (M->pc_off[np] > 0 ? M->pc_off[np] : 1));
  for (int64_t p = 0; p < np; ++p) {
    int64_t o = M->pc_off[p];
    for (int64_t k = 0; k < tf[p]; ++k)
      if (k == 0 || tmp[cnt[p] + k] != tmp[cnt[p] + k - 1]) M->pc_cell[o++] = tmp[cnt[p] + k];
  }
  free(tmp); free(tf); free(cnt);

  /* face centres and area vectors S_f = sum 1/2 (p_i - c_f) x (p_i+1 - c_f) */
  M->S = malloc(sizeof(double) * 3 * nf);
  M->cfc = malloc(sizeof(double) * 3 * nf);
  for (int64_t f = 0; f < nf; ++f) {
    double c[3];
    face_centre(M, f, c);
    memcpy(&M->cfc[3 * f], c, 24);
    double s[3] = {0, 0, 0};
    int64_t b = foff[f], n = foff[f + 1] - b;
    for (int64_t i = 0; i < n; ++i) {
      const double *a = &M->x[3 * (int64_t)fpts[b + i]];
      const double *q = &M->x[3 * (int64_t)fpts[b + (i + 1) % n]];
      double u[3], v[3], w[3];
      v_sub(a, c, u); v_sub(q, c, v); v_cross(u, v, w);
      for (int j = 0; j < 3; ++j) s[j] += 0.5 * w[j];
    }
    memcpy(&M->S[3 * f], s, 24);
  }

  /* cell volume and centroid: tets (mean of cell points, c_f, p_i, p_i+1)
   * READING: the paper leaves the cell centre of eq. 2.7 undefined; the
   * volume centroid is used. */
  M->V = malloc(sizeof(double) * nc);
  M->xc = malloc(sizeof(double) * 3 * nc);
  for (int64_t c = 0; c < nc; ++c) {
    opoly P;
    cell_poly(M, c, &P);
    double xm[3] = {0, 0, 0};
    for (int i = 0; i < P.nv; ++i) for (int j = 0; j < 3; ++j) xm[j] += P.v[i][j];
    for (int j = 0; j < 3; ++j) xm[j] /= P.nv;
    double vol = 0.0, mom[3] = {0, 0, 0};
    for (int64_t k = M->cf_off[c]; k < M->cf_off[c + 1]; ++k) {
      int64_t f = M->cf_face[k];
      int sg = M->cf_sign[k];
      const double *fc = &M->cfc[3 * f];
      int64_t b = foff[f], n = foff[f + 1] - b;
      for (int64_t i = 0; i < n; ++i) {
        const double *a = &M->x[3 * (int64_t)fpts[b + i]];
        const double *q = &M->x[3 * (int64_t)fpts[b + (i + 1) % n]];
        double t = sg * tet6(xm, fc, a, q) / 6.0;
        vol += t;
        for (int j = 0; j < 3; ++j) mom[j] += t * (xm[j] + fc[j] + a[j] + q[j]) / 4.0;
      }
    }
    M->V[c] = vol;
    for (int j = 0; j < 3; ++j) M->xc[3 * c + j] = mom[j] / vol;
  }

  /* inverse-distance weights of the point-cells (eqs. 2.6-2.7) */
  M->w_pc = malloc(sizeof(double) * (M->pc_off[np] > 0 ? M->pc_off[np] : 1));
  for (int64_t p = 0; p < np; ++p) {
    double sum = 0.0;
    for (int64_t k = M->pc_off[p]; k < M->pc_off[p + 1]; ++k) {
      double r[3];
      v_sub(&M->x[3 * p], &M->xc[3 * (int64_t)M->pc_cell[k]], r);
      M->w_pc[k] = 1.0 / v_norm(r);
      sum += M->w_pc[k];
    }
    for (int64_t k = M->pc_off[p]; k < M->pc_off[p + 1]; ++k) M->w_pc[k] /= sum;
  }

  /* flux stencil of a face: the point-cells of its points (Section 2.3: the
   * stencil must contain point and edge neighbours) */
  M->st_off = calloc(nf + 1, sizeof(int64_t));
  int32_t *buf = malloc(sizeof(int32_t) * 4096);
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t f = 0; f < nf; ++f) {
      int nb = 0;
      for (int64_t k = foff[f]; k < foff[f + 1]; ++k) {
        int64_t p = fpts[k];
        for (int64_t j = M->pc_off[p]; j < M->pc_off[p + 1]; ++j)
          if (nb < 4096) buf[nb++] = M->pc_cell[j];
      }
      qsort(buf, nb, sizeof(int32_t), cmp_i32);
      int u = 0;
      for (int k = 0; k < nb; ++k)
        if (k == 0 || buf[k] != buf[k - 1]) {
          if (pass == 1) M->st_cell[M->st_off[f] + u] = buf[k];
          ++u;
        }
      if (pass == 0) M->st_off[f + 1] = u;
    }
    if (pass == 0) {
      for (int64_t f = 0; f < nf; ++f) M->st_off[f + 1] += M->st_off[f];
      M->st_cell = malloc(sizeof(int32_t) * (M->st_off[nf] > 0 ? M->st_off[nf] : 1));
    }
  }
  free(buf);

  M->Up = calloc(3 * np, sizeof(double));
  M->F0 = calloc(nf, sizeof(double));
  M->cls = calloc(nc, 1);
  M->pn = calloc(3 * nc, sizeof(double));
  M->ps = calloc(nc, sizeof(double));
  M->grad = calloc(3 * nc, sizeof(double));
  return M;
}

void orc_destroy(omesh *M) {
  if (!M) return;
  free(M->x); free(M->foff); free(M->fpts); free(M->own); free(M->nei);
  free(M->cf_off); free(M->cf_face); free(M->cf_sign); free(M->pc_off); free(M->pc_cell);
  free(M->w_pc); free(M->st_off); free(M->st_cell); free(M->V); free(M->xc); free(M->S);
  free(M->cfc); free(M->Up); free(M->F0); free(M->cls); free(M->pn); free(M->ps); free(M->grad);
  free(M);
}

void orc_set_eps(omesh *M, double eps) { M->eps = eps; }

/* OpenMP threads of the following calls (n <= 0: leave as is); returns the
 * number in use before the call.  For timing the oracle on fewer cores. */
int orc_set_threads(int n) {
  int before = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return before;
}
/* gradient of the reconstruction: 0 NAG, 1 generalized LSQ */
void orc_set_gradient(omesh *M, int kind) { M->grad_kind = kind; }

/* geometry getters for the tests */
void orc_geometry(const omesh *M, double *V, double *xc, double *S, double *cf) {
  if (V) memcpy(V, M->V, sizeof(double) * M->nc);
  if (xc) memcpy(xc, M->xc, sizeof(double) * 3 * M->nc);
  if (S) memcpy(S, M->S, sizeof(double) * 3 * M->nf);
  if (cf) memcpy(cf, M->cfc, sizeof(double) * 3 * M->nf);
}
int64_t orc_stencil_size(const omesh *M) { return M->st_off[M->nf]; }
void orc_stencil(const omesh *M, int64_t *off, int32_t *cells) {
  memcpy(off, M->st_off, sizeof(int64_t) * (M->nf + 1));
  memcpy(cells, M->st_cell, sizeof(int32_t) * M->st_off[M->nf]);
}

/* ------------------------------------------------------------------ */
/* point velocity by IDW (eqs. 2.6-2.7, applied to U in Section 2.3)   */
/* ------------------------------------------------------------------ */
void orc_set_velocity(omesh *M, const double *Uc, const double *F0, double *Up_out) {
  memcpy(M->F0, F0, sizeof(double) * M->nf);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < M->np; ++p) {
    double u[3] = {0, 0, 0};
    for (int64_t k = M->pc_off[p]; k < M->pc_off[p + 1]; ++k)
      for (int j = 0; j < 3; ++j) u[j] += M->w_pc[k] * Uc[3 * (int64_t)M->pc_cell[k] + j];
    memcpy(&M->Up[3 * p], u, 24);
  }
  if (Up_out) memcpy(Up_out, M->Up, sizeof(double) * 3 * M->np);
}

/* ------------------------------------------------------------------ */
/* flux polyhedron (eq. 2.16, tetrahedral decomposition eq. 2.18)      */
/* ------------------------------------------------------------------ */
/* READING: the correction shifts the swept end points along the point
 * velocity directions; one factor lambda per face scales every sweep vector
 * of that face, so the swept point of face point p is x_p - lambda * s * dt * U_p.
 * The polyhedron surface is: base fan (c_f, p_i, p_i+1), top fan
 * (c_q, q_i+1, q_i) about the mean c_q of the swept points, and each side
 * quad (p_i+1, p_i, q_i, q_i+1) split into four triangles about its vertex
 * mean.  Its tetrahedra have apex c_f; the base ones vanish. */
typedef struct {
  int n;                        /* number of face points           */
  int nt;                       /* number of tets (5 n)            */
  double apex[3];
  double t[5 * O_MAXN][3][3];   /* the three other vertices       */
} oflux;

static void flux_polyhedron(const omesh *M, int64_t f, double dt, double s, double lam,
                            oflux *X) {
  int64_t b = M->foff[f];
  int n = (int)(M->foff[f + 1] - b);
  double p[O_MAXN][3], q[O_MAXN][3], cq[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const double *xp = &M->x[3 * (int64_t)M->fpts[b + i]];
    const double *up = &M->Up[3 * (int64_t)M->fpts[b + i]];
    for (int j = 0; j < 3; ++j) {
      p[i][j] = xp[j];
      q[i][j] = xp[j] - lam * s * dt * up[j];      /* eq. 2.16 */
      cq[j] += q[i][j] / n;
    }
  }
  X->n = n;
  memcpy(X->apex, &M->cfc[3 * f], 24);
  int k = 0;
  for (int i = 0; i < n; ++i) {
    int i1 = (i + 1) % n;
    double m[3];
    for (int j = 0; j < 3; ++j) m[j] = 0.25 * (p[i][j] + p[i1][j] + q[i][j] + q[i1][j]);
    /* top triangle */
    memcpy(X->t[k][0], cq, 24); memcpy(X->t[k][1], q[i1], 24); memcpy(X->t[k][2], q[i], 24); ++k;
    /* side quad (p_i+1, p_i, q_i, q_i+1) about its mean */
    memcpy(X->t[k][0], m, 24); memcpy(X->t[k][1], p[i1], 24); memcpy(X->t[k][2], p[i], 24); ++k;
    memcpy(X->t[k][0], m, 24); memcpy(X->t[k][1], p[i], 24); memcpy(X->t[k][2], q[i], 24); ++k;
    memcpy(X->t[k][0], m, 24); memcpy(X->t[k][1], q[i], 24); memcpy(X->t[k][2], q[i1], 24); ++k;
    memcpy(X->t[k][0], m, 24); memcpy(X->t[k][1], q[i1], 24); memcpy(X->t[k][2], p[i1], 24); ++k;
  }
  X->nt = k;
}

/* V_{f,S}: sum of the signed tet volumes (eqs. 2.18-2.19 times dt). */
static double flux_volume(const oflux *X) {
  double v = 0.0;
  for (int k = 0; k < X->nt; ++k) v += tet6(X->apex, X->t[k][0], X->t[k][1], X->t[k][2]);
  return v / 6.0;
}

double orc_flux_volume(const omesh *M, int64_t f, double dt, double s, double lam) {
  oflux X;
  flux_polyhedron(M, f, dt, s, lam, &X);
  return flux_volume(&X);
}

/* Flux correction (Section 2.3): the swept polyhedron is corrected by the
 * secant method until its volume equals F_f dt (eq. 2.17 with the sign of
 * F_f, eqs. 2.20-2.21), moving the end points along the point trajectories
 * without topology changes.
 * READING: one factor lambda per face scales every sweep vector of the face.
 * Every swept vertex is affine in lambda, so V(lambda) is exactly a cubic;
 * the monotone branch of V through lambda = 0 is bounded by the real roots
 * of V' nearest to 0, located from the cubic through the direct samples
 * V(0) = 0, V(1), V(2), V(3).  The root is sought on the side of 0 where V
 * takes the sign of F dt.  Secant iterates start from lambda = 0 and the
 * plain sweep (lambda = +-1), inside that bracket; an iterate leaving the
 * bracket is replaced by bisection.  Converged when |V - F dt| <= 1e-14 |F dt|
 * or the bracket is exhausted.
 * If F dt lies beyond the extremum of V at the branch end, lambda is set to
 * that extremum or to the plain sweep (+-1 on the same side), whichever is
 * nearer to 0, and status 1 is returned; such a face carries its
 * polyhedron's phase fraction of F dt, or the donor cell's (see
 * phase_flux_face). */
static void branch_cubic(const omesh *M, int64_t f, double dt, double s, double *a1,
                         double *a2, double *a3) {
  double V1 = orc_flux_volume(M, f, dt, s, 1.0);
  double V2 = orc_flux_volume(M, f, dt, s, 2.0);
  double V3 = orc_flux_volume(M, f, dt, s, 3.0);
  *a3 = (V3 - 3.0 * V2 + 3.0 * V1) / 6.0;
  *a2 = (V2 - 2.0 * V1 - 6.0 * *a3) / 2.0;
  *a1 = V1 - *a2 - *a3;
}

/* first root of a1 + 2 a2 t + 3 a3 t^2 with t > 0 (INFINITY if none); the
 * two roots are taken as q / (3 a3) and a1 / q with q = -(a2 + sgn(a2) sqrt D),
 * which avoids cancellation when a3 is small */
static double first_positive_root(double a1, double a2, double a3) {
  double te = INFINITY;
  if (a3 != 0.0) {
    double disc = a2 * a2 - 3.0 * a1 * a3;
    if (disc >= 0.0) {
      double q = -(a2 + copysign(sqrt(disc), a2));
      double r1 = q / (3.0 * a3), r2 = (q != 0.0) ? a1 / q : r1;
      if (r1 > 0.0) te = fmin(te, r1);
      if (r2 > 0.0) te = fmin(te, r2);
    }
  } else if (a2 != 0.0) {
    double r = -a1 / (2.0 * a2);
    if (r > 0.0) te = r;
  }
  return te;
}

static int correct_face(const omesh *M, int64_t f, double dt, double s, double *lam_out,
                        int *iters) {
  double target = s * M->F0[f] * dt;
  *iters = 0;
  *lam_out = 0.0;
  if (target == 0.0) return 0;
  double a1, a2, a3;
  branch_cubic(M, f, dt, s, &a1, &a2, &a3);
  if (!(a1 != 0.0)) return 1;
  /* side of 0 on which V takes the sign of the target; in t = lambda / dir
   * the cubic is b1 t + b2 t^2 + b3 t^3 with b1 > 0 on the branch */
  double dir = ((a1 > 0.0) == (target > 0.0)) ? 1.0 : -1.0;
  double te = first_positive_root(a1 * dir, a2, a3 * dir);
  double end = isfinite(te) ? fmin(te, 32.0) : 32.0;
  double vend = orc_flux_volume(M, f, dt, s, dir * end);
  if ((vend - target) * (target > 0 ? 1.0 : -1.0) < 0.0) {
    *lam_out = dir * fmin(end, 1.0);
    return 1;
  }
  /* bracket [lo, hi] around the root, g(lo) and g(hi) of opposite sign */
  double lo = fmin(0.0, dir * end), hi = fmax(0.0, dir * end);
  double glo = (lo == 0.0) ? -target : vend - target;
  /* secant iterates from (0, -target) and (dir, V(dir) - target) */
  double x0 = 0.0, g0 = -target;
  double x1 = dir, g1 = orc_flux_volume(M, f, dt, s, dir) - target;
  double x = x1;
  if (fabs(g1) <= 1e-14 * fabs(target) && x1 > lo && x1 < hi) { *lam_out = x1; return 0; }
  int bisect = 0;
  for (int it = 0; it < 200; ++it) {
    double xn;
    if (!bisect && g1 != g0) {
      xn = x1 - g1 * (x1 - x0) / (g1 - g0);
      if (!(xn > lo && xn < hi)) { bisect = 1; xn = 0.5 * (lo + hi); }
    } else {
      xn = 0.5 * (lo + hi);
    }
    double gn = orc_flux_volume(M, f, dt, s, xn) - target;
    ++*iters;
    x = xn;
    if (fabs(gn) <= 1e-14 * fabs(target)) break;
    if ((gn < 0.0) == (glo < 0.0)) { lo = xn; glo = gn; } else { hi = xn; }
    x0 = x1; g0 = g1; x1 = xn; g1 = gn;
    if (hi - lo <= 4e-16 * fmax(fabs(lo), fabs(hi))) break;
  }
  *lam_out = x;
  return 0;
}

/* lambda, iteration count and status for every face */
int64_t orc_flux_correction(const omesh *M, double dt, double s, double *lam, int32_t *iters,
                            int8_t *status) {
  int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
  for (int64_t f = 0; f < M->nf; ++f) {
    int it = 0;
    int st = correct_face(M, f, dt, s, &lam[f], &it);
    if (iters) iters[f] = it;
    if (status) status[f] = (int8_t)st;
    bad += st;
  }
  return bad;
}

/* ------------------------------------------------------------------ */
/* reconstruction: Algorithm 1                                         */
/* ------------------------------------------------------------------ */
/* Volume of cell c below the plane n.x <= s by clipping and capping. */
static double cell_cut_volume(const omesh *M, int64_t c, const double *n, double s) {
  opoly P;
  cell_poly(M, c, &P);
  opoly_clip(&P, n, s);
  return opoly_volume(&P);
}

/* NAG gradient (Section 2.2.1): IDW cell -> point values (eq. 2.6), face
 * value as the area-weighted mean of fan-triangle averages (eqs. 2.8-2.11),
 * Gauss gradient (eq. 2.12). */
static void nag_gradient(const omesh *M, int64_t c, const double *alpha, const double *ap,
                         double *g) {
  g[0] = g[1] = g[2] = 0.0;
  for (int64_t k = M->cf_off[c]; k < M->cf_off[c + 1]; ++k) {
    int64_t f = M->cf_face[k];
    int sg = M->cf_sign[k];
    int64_t b = M->foff[f], n = M->foff[f + 1] - b;
    double fprime = 0.0;
    for (int64_t i = 0; i < n; ++i) fprime += ap[M->fpts[b + i]];
    fprime /= (double)n;                                   /* eq. 2.8 */
    const double *fc = &M->cfc[3 * f];
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t pa = M->fpts[b + i], pb = M->fpts[b + (i + 1) % n];
      double u[3], v[3], w[3];
      v_sub(&M->x[3 * pa], fc, u); v_sub(&M->x[3 * pb], fc, v); v_cross(u, v, w);
      double At = 0.5 * v_norm(w);                         /* triangle area */
      double phit = (fprime + ap[pa] + ap[pb]) / 3.0;      /* eq. 2.11 */
      num += At * phit;
      den += At;
    }
    double af = num / den;                                 /* eqs. 2.9-2.10 */
    for (int j = 0; j < 3; ++j) g[j] += sg * af * M->S[3 * f + j];
  }
  (void)alpha;
  for (int j = 0; j < 3; ++j) g[j] /= M->V[c];            /* eq. 2.12 */
}

/* The cells other than c that share a point with c, each once, in
 * ascending order (the point neighbours of Sections 2.2.1 and 2.3).  The
 * caller frees the list. */
static int32_t *point_neighbours(const omesh *M, int64_t c, int64_t *count) {
  int32_t *nb = NULL;
  int64_t nn = 0, cap = 0;
  for (int64_t k = M->cf_off[c]; k < M->cf_off[c + 1]; ++k) {
    int64_t f = M->cf_face[k];
    for (int64_t i = M->foff[f]; i < M->foff[f + 1]; ++i) {
      int64_t p = M->fpts[i];
      for (int64_t j = M->pc_off[p]; j < M->pc_off[p + 1]; ++j) {
        if (M->pc_cell[j] == c) continue;
        if (nn == cap) {
          cap = cap ? 2 * cap : 64;
          nb = realloc(nb, sizeof(int32_t) * cap);
        }
        nb[nn++] = M->pc_cell[j];
      }
    }
  }
  if (nn > 1) qsort(nb, nn, sizeof(int32_t), cmp_i32);
  int64_t u = 0;
  for (int64_t i = 0; i < nn; ++i)
    if (u == 0 || nb[i] != nb[u - 1]) nb[u++] = nb[i];
  *count = u;
  return nb;
}

/* Generalized least-squares gradient (Section 2.2.1, after the NAG
 * gradient): over the point neighbours k of cell c (the cells sharing a point
 * with it), minimise sum_k w_ck^2 E_ck^2 with E_ck = -(phi_c - phi_k) +
 * g . (x_c - x_k) and w_ck the inverse distance of the centroids.  The normal
 * equations (sum w^2 d d^T) g = sum w^2 d (phi_k - phi_c), d = x_k - x_c, are
 * a 3x3 system, solved here by Cramer's rule. */
static void lsq_gradient(const omesh *M, int64_t c, const double *phi, double *g) {
  int64_t nn = 0;
  int32_t *nb = point_neighbours(M, c, &nn);
  double A[3][3] = {{0}}, b[3] = {0};
  for (int64_t i = 0; i < nn; ++i) {
    int64_t k = nb[i];
    double d[3];
    v_sub(&M->xc[3 * k], &M->xc[3 * c], d);
    double w2 = 1.0 / v_dot(d, d);                 /* w_ck^2, w = 1/|d| */
    double dphi = phi[k] - phi[c];
    for (int r = 0; r < 3; ++r) {
      b[r] += w2 * d[r] * dphi;
      for (int q = 0; q < 3; ++q) A[r][q] += w2 * d[r] * d[q];
    }
  }
  free(nb);
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
               A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  for (int r = 0; r < 3; ++r) {
    double Ar[3][3];
    memcpy(Ar, A, sizeof A);
    for (int q = 0; q < 3; ++q) Ar[q][r] = b[q];     /* column r replaced by b */
    double dr = Ar[0][0] * (Ar[1][1] * Ar[2][2] - Ar[1][2] * Ar[2][1]) -
                Ar[0][1] * (Ar[1][0] * Ar[2][2] - Ar[1][2] * Ar[2][0]) +
                Ar[0][2] * (Ar[1][0] * Ar[2][1] - Ar[1][1] * Ar[2][0]);
    g[r] = det != 0.0 ? dr / det : 0.0;
  }
}

static void cell_gradient(const omesh *M, int64_t c, const double *alpha, const double *ap,
                          double *g) {
  if (M->grad_kind == 1) lsq_gradient(M, c, alpha, g);
  else nag_gradient(M, c, alpha, ap, g);
}

/* Interface positioning (Section 2.2.2, Algorithm 1): the fill level
 * g(s) = |C ∩ {n.x <= s}| / V_c - alpha rises monotonically from -alpha to
 * 1 - alpha over [min n.x_v, max n.x_v]; secant iterations, and once the
 * secant diverges (two arguments outside the search interval) bisection.
 * READING: converged when |g| <= 1e-15 or the interval is down to a few ulp. */
static double position_plane(const omesh *M, int64_t c, const double *n, double alpha,
                             int *iters) {
  opoly P;
  cell_poly(M, c, &P);
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < P.nv; ++i) {
    double h = v_dot(n, P.v[i]);
    if (h < lo) lo = h;
    if (h > hi) hi = h;
  }
  double V = M->V[c];
  double s0 = lo, g0 = -alpha, s1 = hi, g1 = 1.0 - alpha;
  double glo = g0;
  int outside = 0, bisect = 0;
  double s = 0.5 * (lo + hi);
  *iters = 0;
  for (int it = 0; it < 300; ++it) {
    double sn;
    if (!bisect && g1 != g0) {
      sn = s1 - g1 * (s1 - s0) / (g1 - g0);
      if (!(sn > lo && sn < hi)) {
        ++outside;
        if (outside >= 2) bisect = 1;
        sn = 0.5 * (lo + hi);
      }
    } else {
      sn = 0.5 * (lo + hi);
    }
    double gn = cell_cut_volume(M, c, n, sn) / V - alpha;
    ++*iters;
    s = sn;
    if (fabs(gn) <= 1e-15) break;
    if ((gn < 0.0) == (glo < 0.0)) { lo = sn; glo = gn; } else { hi = sn; }
    s0 = s1; g0 = g1; s1 = sn; g1 = gn;
    if (hi - lo <= 4e-16 * fmax(1.0, fmax(fabs(lo), fabs(hi)))) break;
  }
  return s;
}

/* Algorithm 1 over the mesh.  Classes: 0 empty (alpha <= eps), 2 full
 * (alpha >= 1 - eps), 1 interface; 3 = interface cell with a vanishing
 * gradient (READING: |grad alpha| h_c < 1e-8, treated as homogeneous with
 * its volume fraction).  Outputs may be NULL. */
int64_t orc_reconstruct(omesh *M, const double *alpha, int8_t *cls, double *grad,
                        double *nrm, double *spos, int32_t *iters) {
  double *ap = malloc(sizeof(double) * M->np);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < M->np; ++p) {
    double a = 0.0;
    for (int64_t k = M->pc_off[p]; k < M->pc_off[p + 1]; ++k)
      a += M->w_pc[k] * alpha[M->pc_cell[k]];
    ap[p] = a;                                             /* eq. 2.6 */
  }
  int64_t nint = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nint)
  for (int64_t c = 0; c < M->nc; ++c) {
    double a = alpha[c];
    int it = 0;
    M->pn[3 * c] = M->pn[3 * c + 1] = M->pn[3 * c + 2] = 0.0;
    M->ps[c] = 0.0;
    M->grad[3 * c] = M->grad[3 * c + 1] = M->grad[3 * c + 2] = 0.0;
    if (a <= M->eps) M->cls[c] = 0;
    else if (a >= 1.0 - M->eps) M->cls[c] = 2;
    else {
      double g[3];
      cell_gradient(M, c, alpha, ap, g);
      memcpy(&M->grad[3 * c], g, 24);
      double gn = v_norm(g);
      double hc = cbrt(M->V[c]);
      if (gn * hc < 1e-8) {
        M->cls[c] = 3;
      } else {
        double n[3] = {-g[0] / gn, -g[1] / gn, -g[2] / gn};
        memcpy(&M->pn[3 * c], n, 24);
        M->ps[c] = position_plane(M, c, n, a, &it);
        M->cls[c] = 1;
        ++nint;
      }
    }
    if (iters) iters[c] = it;
  }
  free(ap);
  if (cls) memcpy(cls, M->cls, M->nc);
  if (grad) memcpy(grad, M->grad, sizeof(double) * 3 * M->nc);
  if (nrm) memcpy(nrm, M->pn, sizeof(double) * 3 * M->nc);
  if (spos) memcpy(spos, M->ps, sizeof(double) * M->nc);
  return nint;
}

/* ------------------------------------------------------------------ */
/* fluxed phase volume (eqs. 2.22-2.23)                                */
/* ------------------------------------------------------------------ */
/* |T ∩ C_c| and |T ∩ C_c ∩ I+| for a tet T: clip the tet by every face
 * plane of cell c (outward normal S_f, through the face centre), then by the
 * PLIC plane when the cell is an interface cell. */
static int tet_cell_volumes(const omesh *M, const double *a, const double *b, const double *c,
                            const double *d, int64_t cell, double *vcell, double *vphase) {
  opoly P;
  opoly_tet(&P, a, b, c, d);
  int err = 0;
  for (int64_t k = M->cf_off[cell]; k < M->cf_off[cell + 1] && P.nv; ++k) {
    int64_t f = M->cf_face[k];
    int sg = M->cf_sign[k];
    double n[3] = {sg * M->S[3 * f], sg * M->S[3 * f + 1], sg * M->S[3 * f + 2]};
    double s = v_dot(n, &M->cfc[3 * f]);
    err |= opoly_clip(&P, n, s);
  }
  *vcell = opoly_volume(&P);
  int cl = M->cls[cell];
  if (cl == 2) *vphase = *vcell;
  else if (cl == 0) *vphase = 0.0;
  else if (cl == 3) *vphase = -1.0;        /* caller weights by alpha */
  else {
    err |= opoly_clip(&P, &M->pn[3 * cell], M->ps[cell]);
    *vphase = opoly_volume(&P);
  }
  return err;
}

/* Phase volume of face f for the last reconstruction.
 * kind: 0 no flux, 1 trivially empty stencil, 2 trivially full stencil,
 *       3 geometric, 4 correction target unreachable and the clamped
 *       polyhedron below a quarter of F dt (donor cell).
 * READING: outside the domain counts as empty; for a boundary face the
 * full-stencil shortcut is not taken (its polyhedron may lie outside).
 * Returns the stencil leak |sum_c sum_k sgn_k |T_k ∩ C_c| - V_f| relative to
 * max(sum_k |T_k|, V_owner) when check_leak is set (geometric faces only).
 * Volume outside the domain counts as leaked. */
static double phase_flux_face(const omesh *M, int64_t f, double dt, double s, double lam,
                              int status, const double *alpha, int check_leak, double *vphase,
                              int *kind, int *err) {
  *err = 0;
  double F = s * M->F0[f];
  if (F == 0.0) { *vphase = 0.0; *kind = 0; return 0.0; }
  int any_nonempty = 0, all_full = 1;
  for (int64_t k = M->st_off[f]; k < M->st_off[f + 1]; ++k) {
    int cl = M->cls[M->st_cell[k]];
    if (cl != 0) any_nonempty = 1;
    if (cl != 2) all_full = 0;
  }
  if (!any_nonempty) { *vphase = 0.0; *kind = 1; return 0.0; }
  if (all_full && f < M->ni) { *vphase = F * dt; *kind = 2; return 0.0; }
  if (status == 1) {
    /* READING (the paper's correction always converges; an unreachable
     * target is not treated): no swept polyhedron on the branch has volume
     * F dt.  If the clamped polyhedron still holds at least a quarter of
     * F dt, on its side, its phase fraction is applied to F dt (the scalar
     * coefficient correction the paper cites, Section 2.3; the scale is then
     * at most 4); otherwise it is too small to say anything and the face
     * carries the upwind (donor) cell's fraction of F dt, the cell the flux
     * leaves (outside the domain is empty). */
    double vl = orc_flux_volume(M, f, dt, s, lam);
    if (!(fabs(vl) >= 0.25 * fabs(F * dt) && vl * F > 0.0)) {
      int64_t donor = F > 0.0 ? M->own[f] : (f < M->ni ? M->nei[f] : -1);
      *vphase = donor >= 0 ? alpha[donor] * (F * dt) : 0.0;
      *kind = 4;
      return 0.0;
    }
  }
  *kind = 3;
  oflux X;
  flux_polyhedron(M, f, dt, s, lam, &X);
  double total = 0.0, covered = 0.0, vf = 0.0, gross = 0.0;
  for (int t = 0; t < X.nt; ++t) {
    double det = tet6(X.apex, X.t[t][0], X.t[t][1], X.t[t][2]);
    if (det == 0.0) continue;
    vf += det / 6.0;
    gross += fabs(det) / 6.0;
    double sgn = det > 0 ? 1.0 : -1.0;
    const double *a = X.apex, *b = X.t[t][0], *c = det > 0 ? X.t[t][1] : X.t[t][2],
                 *d = det > 0 ? X.t[t][2] : X.t[t][1];
    for (int64_t k = M->st_off[f]; k < M->st_off[f + 1]; ++k) {
      int64_t cell = M->st_cell[k];
      int cl = M->cls[cell];
      if (cl == 0 && !check_leak) continue;
      double vc, vp;
      *err |= tet_cell_volumes(M, a, b, c, d, cell, &vc, &vp);
      covered += sgn * vc;
      if (cl == 3) vp = alpha[cell] * vc;
      total += sgn * vp;
    }
  }
  /* a clamped face: the phase fraction of its polyhedron times F dt */
  if (status == 1 && vf != 0.0) total *= (F * dt) / vf;
  *vphase = total;
  /* uncovered signed volume relative to the gross tet volume of the face or
   * the owner cell's volume, whichever is larger */
  double ref = fmax(gross, M->V[M->own[f]]);
  return check_leak ? fabs(covered - vf) / ref : 0.0;
}

/* V_{f,alpha} for every face.  Outputs may be NULL.  Returns the number of
 * geometric faces; *max_leak receives the largest stencil leak relative to
 * the gross tet volume of its face. */
int64_t orc_phase_flux(const omesh *M, double dt, double s, const double *lam,
                       const int8_t *status, const double *alpha, int check_leak,
                       double *vphase, int8_t *kind, double *max_leak, int64_t *nerr) {
  int64_t ngeo = 0, ne = 0;
  double leak = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : ngeo, ne) reduction(max : leak)
  for (int64_t f = 0; f < M->nf; ++f) {
    int kd = 0, er = 0;
    double v = 0.0;
    double l = phase_flux_face(M, f, dt, s, lam[f], status ? status[f] : 0, alpha, check_leak,
                               &v, &kd, &er);
    if (vphase) vphase[f] = v;
    if (kind) kind[f] = (int8_t)kd;
    if (kd == 3) {
      ++ngeo;
      if (l > leak) leak = l;
    }
    ne += er;
  }
  if (max_leak) *max_leak = leak;
  if (nerr) *nerr = ne;
  return ngeo;
}

/* ------------------------------------------------------------------ */
/* conservative update (eq. 2.2 with eq. 2.5; outflow-only phase volume) */
/* ------------------------------------------------------------------ */
/* READING (Section 2.3, narrow band): a bulk cell is one whose volume
 * fraction gradient vanishes; taken here as a cell such that it and every
 * cell sharing a point with it hold alpha exactly 0, or all exactly 1.  Then
 * every inverse-distance point value of the cell equals its alpha and the NAG
 * gradient is zero in exact arithmetic. */
static int bulk_cell(const omesh *M, int64_t c, const double *alpha) {
  const double a = alpha[c];
  if (a != 0.0 && a != 1.0) return 0;
  int64_t nn = 0;
  int32_t *nb = point_neighbours(M, c, &nn);
  int bulk = 1;
  for (int64_t i = 0; i < nn && bulk; ++i) bulk = alpha[nb[i]] == a;
  free(nb);
  return bulk;
}

void orc_bulk_cells(const omesh *M, const double *alpha, int8_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < M->nc; ++c) out[c] = (int8_t)bulk_cell(M, c, alpha);
}

/* alpha_c^{n+1} = alpha_c^n - (1/V_c) sum_f sgn_cf V_{f,alpha}, every cell
 * (with the narrow band: every cell but the bulk cells, whose alpha is left
 * as it is; the paper computes the phase volumes of their faces all the same),
 * no clamping.  Returns the boundary ledger sum of V_{f,alpha} over boundary
 * faces (volume that left the domain, negative for inflow). */
double orc_update(const omesh *M, const double *alpha, const double *vphase, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < M->nc; ++c) {
    if (M->band && bulk_cell(M, c, alpha)) {
      out[c] = alpha[c];
      continue;
    }
    double acc = 0.0;
    for (int64_t k = M->cf_off[c]; k < M->cf_off[c + 1]; ++k)
      acc += M->cf_sign[k] * vphase[M->cf_face[k]];
    out[c] = alpha[c] - acc / M->V[c];
  }
  double B = 0.0;
  for (int64_t f = M->ni; f < M->nf; ++f) B += vphase[f];
  return B;
}

/* ------------------------------------------------------------------ */
/* wisp redistribution (Section 2.3)                                    */
/* ------------------------------------------------------------------ */
/* Wisps, small volume fractions left outside the interface band by the
 * update, are moved conservatively to the interface cells around them, and
 * no receiving cell may be pushed out of the interface band (no new over- or
 * undershoot and no new wisp).  The paper cites Harvie and Fletcher and
 * gives no formulas; READING, step by step:
 *   - wisp: a cell whose alpha lies outside the band (eps, 1 - eps) but is
 *     not exactly 0 or 1 (phase wisps 0 < alpha <= eps, void wisps
 *     1 - eps <= alpha < 1, undershoots alpha < 0, overshoots alpha > 1);
 *     its signed excess is m_w = (alpha_w - t) V_w with the target t = 0 if
 *     alpha_w <= eps, else 1;
 *   - receivers: interface cells (eps < alpha < 1 - eps) sharing a point with
 *     the wisp;
 *   - a receiver r can take (1 - eps - alpha_r) V_r of phase and give
 *     (alpha_r - eps) V_r; it offers each wisp around it the share of that
 *     room (for m > 0) or store (for m < 0) proportional to |m_w| among the
 *     wisps of the same sign around it;
 *   - a wisp moves min(|m_w|, total offered) and splits it over its receivers
 *     in proportion to their offers; a wisp moved whole is set to its
 *     target exactly, one with too little room around it keeps the rest.
 * All quantities come from the alpha after the update (one pass per step),
 * so every receiver stays within [eps, 1 - eps]: its gain is at most its
 * room and its loss at most its store.  counts: wisps, wisps left with a
 * remainder, receivers. */
void orc_redistribute(const omesh *M, double *alpha, int64_t *counts) {
  const int64_t nc = M->nc;
  const double eps = M->eps;
  double *m = calloc(nc, sizeof(double));      /* signed excess of each wisp */
  double *dpos = calloc(nc, sizeof(double));   /* per receiver: sum of m > 0 around it */
  double *dneg = calloc(nc, sizeof(double));   /*               sum of -m, m < 0 */
  double *moved = calloc(nc, sizeof(double));  /* per wisp: volume moved */
  double *offered = calloc(nc, sizeof(double));
  double *gain = calloc(nc, sizeof(double));
  int8_t *band = malloc(nc);
  int64_t nw = 0, nleft = 0, nrecv = 0;
  for (int64_t c = 0; c < nc; ++c) {
    const double a = alpha[c];
    band[c] = a > eps && a < 1.0 - eps;
    if (!band[c] && a != 0.0 && a != 1.0) {
      m[c] = (a - (a <= eps ? 0.0 : 1.0)) * M->V[c];
      ++nw;
    }
  }
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nrecv)
  for (int64_t r = 0; r < nc; ++r) {
    if (!band[r]) continue;
    int64_t nn = 0;
    int32_t *nb = point_neighbours(M, r, &nn);
    int any = 0;
    for (int64_t i = 0; i < nn; ++i) {
      const double mw = m[nb[i]];
      if (mw > 0.0) dpos[r] += mw;
      if (mw < 0.0) dneg[r] -= mw;
      any |= mw != 0.0;
    }
    nrecv += any;
    free(nb);
  }
  /* the offer of receiver r to wisp w */
#define OFFER(r, w)                                                                    \
  (m[w] > 0.0 ? (1.0 - eps - alpha[r]) * M->V[r] * (m[w] / dpos[r])                   \
              : (alpha[r] - eps) * M->V[r] * (-m[w] / dneg[r]))
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t w = 0; w < nc; ++w) {
    if (m[w] == 0.0) continue;
    int64_t nn = 0;
    int32_t *nb = point_neighbours(M, w, &nn);
    double O = 0.0;
    for (int64_t i = 0; i < nn; ++i)
      if (band[nb[i]]) O += OFFER(nb[i], w);
    offered[w] = O;
    moved[w] = fmin(fabs(m[w]), O);
    free(nb);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < nc; ++r) {
    if (!band[r]) continue;
    int64_t nn = 0;
    int32_t *nb = point_neighbours(M, r, &nn);
    for (int64_t i = 0; i < nn; ++i) {
      const int64_t w = nb[i];
      if (m[w] == 0.0 || offered[w] == 0.0) continue;
      const double x = moved[w] * (OFFER(r, w) / offered[w]);   /* w -> r */
      gain[r] += m[w] > 0.0 ? x : -x;
    }
    free(nb);
  }
#undef OFFER
  for (int64_t c = 0; c < nc; ++c) {
    if (band[c]) {
      alpha[c] += gain[c] / M->V[c];
    } else if (m[c] != 0.0) {
      if (offered[c] >= fabs(m[c])) {
        alpha[c] = alpha[c] <= eps ? 0.0 : 1.0;
      } else {
        alpha[c] -= (m[c] > 0.0 ? moved[c] : -moved[c]) / M->V[c];
        ++nleft;
      }
    }
  }
  counts[0] = nw;
  counts[1] = nleft;
  counts[2] = nrecv;
  free(m); free(dpos); free(dneg); free(moved); free(offered); free(gain); free(band);
}

void orc_set_band(omesh *M, int band) { M->band = band; }
void orc_set_wisps(omesh *M, int wisps) { M->wisps = wisps; }

/* ------------------------------------------------------------------ */
/* geometric mapping after a mesh change (Section 3, Algorithm 2)       */
/* ------------------------------------------------------------------ */
/* The volume fraction of each cell of the new mesh M is the part of it that
 * the old mesh's reconstruction fills.  For new cell c, map_cell lists the
 * old cells it came from (map_off is CSR over the new cells):
 *   - one old cell o that contains c (c refined from o, or c = o): the
 *     paper intersects o's interface plane with c, so alpha_c =
 *     |C_c ∩ {n_o . x <= s_o}| / V_c for an interface cell o; READING: for
 *     an empty, full or vanishing-gradient cell o, alpha_c = alpha_o (the
 *     old cell's content spread evenly, which keeps the volume exactly);
 *   - several old cells whose union is c (c coarsened from them): READING,
 *     the union of their reconstructed phase volumes, alpha_c =
 *     sum_o alpha_o V_o / V_c (|C_o ∩ I_o| = alpha_o V_o by the
 *     positioning).
 * cls_old, n_old (3 per cell), s_old: the reconstruction of alpha_old on the
 * old mesh (classes 0 empty, 1 interface, 2 full, 3 vanishing gradient). */
void orc_map_alpha(const omesh *M, const int64_t *map_off, const int32_t *map_cell,
                   const double *alpha_old, const double *V_old, const int8_t *cls_old,
                   const double *n_old, const double *s_old, double *alpha_new) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < M->nc; ++c) {
    const int64_t k0 = map_off[c], k1 = map_off[c + 1];
    if (k1 - k0 == 1) {
      const int32_t o = map_cell[k0];
      if (cls_old[o] == 1)
        alpha_new[c] = cell_cut_volume(M, c, &n_old[3 * o], s_old[o]) / M->V[c];
      else
        alpha_new[c] = alpha_old[o];
    } else {
      double v = 0.0;
      for (int64_t k = k0; k < k1; ++k) v += alpha_old[map_cell[k]] * V_old[map_cell[k]];
      alpha_new[c] = v / M->V[c];
    }
  }
}

/* ------------------------------------------------------------------ */
/* time loop: all geometry of step n uses alpha^n (explicit Euler, eq. 2.2) */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n_interface, n_geometric, n_fallback, n_unreached, n_clip_errors;
  double ledger, max_leak, max_corr_residual, mean_secant_iters;
  int64_t n_wisps, n_wisps_left;
} ostats;

int orc_advect(omesh *M, double *alpha, int64_t nsteps, const double *dt, const double *sc,
               int check_leak, ostats *st, double *lam_last, double *vphase_last) {
  double *lam = malloc(sizeof(double) * M->nf);
  int32_t *it = malloc(sizeof(int32_t) * M->nf);
  int8_t *stt = malloc(M->nf);
  double *vp = malloc(sizeof(double) * M->nf);
  double *nxt = malloc(sizeof(double) * M->nc);
  memset(st, 0, sizeof(*st));
  double itsum = 0.0;
  int64_t itcnt = 0;
  for (int64_t n = 0; n < nsteps; ++n) {
    st->n_interface += orc_reconstruct(M, alpha, NULL, NULL, NULL, NULL, NULL);
    for (int64_t c = 0; c < M->nc; ++c) st->n_fallback += (M->cls[c] == 3);
    st->n_unreached += orc_flux_correction(M, dt[n], sc[n], lam, it, stt);
    double res = 0.0;
    for (int64_t f = 0; f < M->nf; ++f) {
      double T = sc[n] * M->F0[f] * dt[n];
      if (T != 0.0 && stt[f] == 0) {
        itsum += it[f]; ++itcnt;
        double r = fabs(orc_flux_volume(M, f, dt[n], sc[n], lam[f]) - T) / fabs(T);
        if (r > res) res = r;
      }
    }
    if (res > st->max_corr_residual) st->max_corr_residual = res;
    double leak = 0.0;
    int64_t ne = 0;
    st->n_geometric += orc_phase_flux(M, dt[n], sc[n], lam, stt, alpha, check_leak, vp, NULL,
                                      &leak, &ne);
    st->n_clip_errors += ne;
    if (leak > st->max_leak) st->max_leak = leak;
    st->ledger += orc_update(M, alpha, vp, nxt);
    if (M->wisps) {
      int64_t wc[3];
      orc_redistribute(M, nxt, wc);
      st->n_wisps += wc[0];
      st->n_wisps_left += wc[1];
    }
    memcpy(alpha, nxt, sizeof(double) * M->nc);
  }
  st->mean_secant_iters = itcnt ? itsum / itcnt : 0.0;
  if (lam_last) memcpy(lam_last, lam, sizeof(double) * M->nf);
  if (vphase_last) memcpy(vphase_last, vp, sizeof(double) * M->nf);
  free(lam); free(it); free(stt); free(vp); free(nxt);
  return 0;
}

/* ------------------------------------------------------------------ */
/* primitive exposed for the tests: a convex polyhedron clipped by a    */
/* list of half-spaces {n_k . x <= s_k}; faces as CSR of vertex indices */
/* ------------------------------------------------------------------ */
double orc_clip_volume(int nv, const double *v, int nf, const int32_t *foff,
                       const int32_t *fidx, int nplanes, const double *planes) {
  opoly P;
  if (nv > O_MAXV || nf > O_MAXF) return NAN;
  P.nv = nv; P.nf = nf;
  for (int i = 0; i < nv; ++i) memcpy(P.v[i], &v[3 * i], 24);
  for (int f = 0; f < nf; ++f) {
    P.fn[f] = foff[f + 1] - foff[f];
    for (int k = 0; k < P.fn[f]; ++k) P.fv[f][k] = fidx[foff[f] + k];
  }
  for (int k = 0; k < nplanes; ++k)
    if (opoly_clip(&P, &planes[4 * k], planes[4 * k + 3])) return NAN;
  return opoly_volume(&P);
}

/* cut volume of a mesh cell (used by the positioning pins) */
double orc_cell_cut_volume(const omesh *M, int64_t c, const double *n, double s) {
  return cell_cut_volume(M, c, n, s);
}

/* tet ∩ cell volumes for the partition-of-unity pin */
double orc_tet_cell_volume(const omesh *M, const double *tet, int64_t cell) {
  double vc, vp;
  double det = tet6(&tet[0], &tet[3], &tet[6], &tet[9]);
  if (det > 0) tet_cell_volumes(M, &tet[0], &tet[3], &tet[6], &tet[9], cell, &vc, &vp);
  else tet_cell_volumes(M, &tet[0], &tet[3], &tet[9], &tet[6], cell, &vc, &vp);
  return vc;
}

/* plane of the last reconstruction / class access for tests */
void orc_set_planes(omesh *M, const int8_t *cls, const double *nrm, const double *spos) {
  memcpy(M->cls, cls, M->nc);
  memcpy(M->pn, nrm, sizeof(double) * 3 * M->nc);
  memcpy(M->ps, spos, sizeof(double) * M->nc);
}

/* point values of a cell field by IDW (eq. 2.6), for the tests */
void orc_point_values(const omesh *M, const double *phi, double *out) {
  for (int64_t p = 0; p < M->np; ++p) {
    double a = 0.0;
    for (int64_t k = M->pc_off[p]; k < M->pc_off[p + 1]; ++k)
      a += M->w_pc[k] * phi[M->pc_cell[k]];
    out[p] = a;
  }
}

/* generalized LSQ gradient of an arbitrary cell field on every cell (tests) */
void orc_lsq_gradient(const omesh *M, const double *phi, double *grad) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < M->nc; ++c) lsq_gradient(M, c, phi, &grad[3 * c]);
}

/* NAG gradient of an arbitrary cell field on every cell (tests) */
void orc_nag_gradient(const omesh *M, const double *phi, double *grad) {
  double *ap = malloc(sizeof(double) * M->np);
  orc_point_values(M, phi, ap);
  for (int64_t c = 0; c < M->nc; ++c) nag_gradient(M, c, phi, ap, &grad[3 * c]);
  free(ap);
}

/* tests: prescribe point velocities directly (bypasses the IDW of eq. 2.6) */
void orc_set_point_velocity(omesh *M, const double *Up, const double *F0) {
  memcpy(M->Up, Up, sizeof(double) * 3 * M->np);
  if (F0) memcpy(M->F0, F0, sizeof(double) * M->nf);
}

/* ------------------------------------------------------------------ */
/* subsets, for checking full-size runs on sampled outputs              */
/* ------------------------------------------------------------------ */
/* classes of every cell; NAG gradient and plane only for the listed cells */
void orc_reconstruct_subset(omesh *M, const double *alpha, int64_t ncells, const int64_t *cells) {
  for (int64_t c = 0; c < M->nc; ++c) {
    double a = alpha[c];
    M->cls[c] = a <= M->eps ? 0 : (a >= 1.0 - M->eps ? 2 : 1);
  }
  double *ap = malloc(sizeof(double) * M->np);
  orc_point_values(M, alpha, ap);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < ncells; ++i) {
    int64_t c = cells[i];
    if (M->cls[c] != 1) continue;
    double g[3];
    cell_gradient(M, c, alpha, ap, g);
    memcpy(&M->grad[3 * c], g, 24);
    double gn = v_norm(g);
    if (gn * cbrt(M->V[c]) < 1e-8) { M->cls[c] = 3; continue; }
    double n[3] = {-g[0] / gn, -g[1] / gn, -g[2] / gn};
    memcpy(&M->pn[3 * c], n, 24);
    int it = 0;
    M->ps[c] = position_plane(M, c, n, alpha[c], &it);
  }
  free(ap);
}

void orc_get_planes(const omesh *M, int8_t *cls, double *nrm, double *spos) {
  if (cls) memcpy(cls, M->cls, M->nc);
  if (nrm) memcpy(nrm, M->pn, sizeof(double) * 3 * M->nc);
  if (spos) memcpy(spos, M->ps, sizeof(double) * M->nc);
}

/* flux correction and phase volume for listed faces (planes of the cells in
 * their stencils must have been reconstructed) */
void orc_faces_subset(const omesh *M, double dt, double s, const double *alpha, int64_t nfaces,
                      const int64_t *faces, double *lam, int32_t *iters, int8_t *status,
                      double *vphase, int8_t *kind) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nfaces; ++i) {
    int64_t f = faces[i];
    int it = 0;
    status[i] = (int8_t)correct_face(M, f, dt, s, &lam[i], &it);
    iters[i] = it;
    int kd = 0, er = 0;
    phase_flux_face(M, f, dt, s, lam[i], status[i], alpha, 0, &vphase[i], &kd, &er);
    kind[i] = (int8_t)kd;
  }
}
