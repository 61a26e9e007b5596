// vof_device.hip -- HIP kernels of the geometric PLIC VoF flux path (gfx950).
//
// One step (explicit Euler, eq. 2.2; every geometric quantity uses alpha^n):
//   k_cell_class   cell classes by the band eps < alpha < 1 - eps, list of
//                  interface cells                                (step 4a)
//   k_point_prep   per point: OR of point-cell classes; IDW point values of
//                  alpha for band points (eq. 2.6)                (step 4b)
//   k_flux         per face: swept points (eq. 2.16), the flux polyhedron's
//                  exact volume cubic, Newton correction to F dt (eq. 2.17),
//                  stencil class -> trivial V_alpha or geometric list (1-3)
//   k_plane        per interface cell: NAG gradient (eqs. 2.8-2.12) and
//                  plane positioning (Section 2.2.2)                 (step 4)
//   k_clip         per (geometric face, flux tet): intersection with the
//                  stencil cells and their PLIC half-spaces (eqs. 2.22-2.23)
//   k_face_sum     per geometric face: signed sum of its tet volumes  (5)
//   k_update       per cell: alpha -= (1/V) sum_f sgn V_alpha (eqs. 2.2, 2.5)
//   k_ledger       boundary phase volume of the step (one block, fixed order)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "geom.hpp"
#include "vof_internal.h"
#include "clip.hpp"

namespace vof {

namespace {

constexpr int kWave = 64;     // wavefront width
constexpr int kBlock = 256;
constexpr int kClipBlock = 64;
constexpr unsigned kFluxGrid = 8192;  // flux kernel blocks at most
constexpr int kFastBlock = 64;   // one wave per block in the register clip
// register clip configurations: queued pairs of two or more planes per tet,
// candidate cells of a face group kept in LDS (CAND / F per face), and
// whether the candidates' bounds are kept in LDS (box cells need them).
// Quad faces (a hex face's stencil: 18 cells) take the first; triangle faces
// of tetrahedral meshes (58 stencil cells, about 7 overlapping cells per
// flux tet) the second, at two waves per SIMD.
constexpr int kFastSlots = 4;
constexpr int kTriSlots = 12, kTriCand = 192;
constexpr int kFastPlanes = 4;   // planes per pair in the register clip (more: general)
constexpr int kTriPlanes = 5;    // the same for triangle faces
constexpr int kFastGrid = 4096;   // blocks claim face groups from a counter
constexpr int kClaim = 2;         // face groups per claim
constexpr int kGroupFaces = 4;    // faces per wavefront group (64 / at least 15 tets)
constexpr int kCandPool = 48;
constexpr int kFacePool = 12;     // staged points of a face group: F * max points <= 64 / 5
constexpr int kPlaneGrid = 2048;  // blocks of four waves, four interface cells per wave
static_assert(kMaxCellPlanes * kMaxFacePoints <= 128, "two fan tetrahedra per lane");
static_assert(kMaxCellPlanes <= 16, "cutting-plane masks are 16 bits");
constexpr int kLedgerBlock = 1024;  // the one block of the ledger's second stage
constexpr int kGenTets = 3;        // deferred tets per wavefront in the general clip
constexpr int kGenLanes = 21;      // lanes per tet (a hex face's stencil is 18 cells)
static_assert(kGenTets * kGenLanes <= 64, "tets of a wavefront");
constexpr int kWispGrid = 2048;    // blocks of the wisp passes (wave-stride over the lists)

__device__ __forceinline__ v3 xyz(double4 a) { return mk3(a.x, a.y, a.z); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__host__ __device__ __forceinline__ int64_t grid_for_dev(int64_t n, int block) {
  return (n + block - 1) / block;
}

// Workgroups are dispatched round-robin over the eight XCDs (block b on XCD
// b % 8), each with its own L2; kernels that give every XCD a contiguous
// range of the work take grids that are multiples of 8.
constexpr int kXcds = 8;

// Append the lanes with `pred` to a list: one atomic per wavefront.  Must be
// reached by every lane of the wavefront.
__device__ __forceinline__ int wave_append(int32_t *counter, bool pred) {
  unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return -1;
  int lane = lane_id();
  int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(mask));
  base = __shfl(base, leader);
  int rank = (int)__popcll(mask & ((1ull << lane) - 1ull));
  return pred ? base + rank : -1;
}
// The step's geometric faces: index i < geo_count runs over the faces of up
// to kSmallFace points (slots 0, 1, ...), then over the larger ones (slots
// nf - 1, nf - 2, ...); na = work[kWGeometric].
__device__ __forceinline__ int geo_count(const DState &s) {
  return s.work[kWGeometric] + s.work[kWGeoLarge];
}
__device__ __forceinline__ int64_t geo_slot(const DMesh &m, int na, int i) {
  return i < na ? (int64_t)i : m.nf - 1 - (int64_t)(i - na);
}
// Register-clip face groups of one mesh: the small faces' groups first
// (tsmall tets per face), then the large faces' (the mesh's 5 * maxn).  The
// list counts are read once: the step's claim counter shares their line.
struct ClipGroups {
  int na, nb, tsmall, nsmall, total;
};
__device__ __forceinline__ ClipGroups clip_groups(const DMesh &m, const DState &s) {
  ClipGroups c;
  c.na = s.work[kWGeometric];
  c.nb = s.work[kWGeoLarge];
  c.tsmall = m.tpf < 5 * kSmallFace ? m.tpf : 5 * kSmallFace;
  const int fs = 64 / c.tsmall, fl = 64 / m.tpf;
  c.nsmall = (c.na + fs - 1) / fs;
  c.total = c.nsmall + (c.nb + fl - 1) / fl;
  return c;
}

// Append the threads with `pred` to a list with one atomic per block (the
// waves' counts are combined in LDS).  Every thread of the block must reach
// it; the block size must be kBlock.
__device__ __forceinline__ int block_append(int32_t *counter, bool pred) {
  __shared__ int wbase[kBlock / 64];
  __shared__ int bbase;
  const unsigned long long mask = __ballot(pred);
  const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
  if (lane == 0) wbase[w] = (int)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) { int c = wbase[i]; wbase[i] = tot; tot += c; }
    bbase = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  const int pos = bbase + wbase[w] + (int)__popcll(mask & ((1ull << lane) - 1ull));
  __syncthreads();  // wbase / bbase are reused by the next call
  return pred ? pos : -1;
}

// Append n items per thread to a list (one atomic per block); returns the
// thread's first position.  Must be reached by every thread of the block.
__device__ __forceinline__ int block_append_n(int32_t *counter, int n) {
  __shared__ int wsum[kBlock / 64];
  __shared__ int bbase;
  const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
  int v = n;  // inclusive scan over the wavefront
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) { int c = wsum[i]; wsum[i] = tot; tot += c; }
    bbase = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  const int pos = bbase + wsum[w] + v - n;
  __syncthreads();  // wsum / bbase are reused by the next call
  return pos;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ void wave_count(unsigned long long *dst, unsigned long long v) {
  v = wave_sum(v);
  if (lane_id() == 0 && v) atomicAdd(dst, v);
}

__device__ __forceinline__ void flag(uint32_t *flags, uint32_t bit) { atomicOr(flags, bit); }

// this block's slot of counter id
__device__ __forceinline__ unsigned long long *cnt_at(unsigned long long *cnt, int id) {
  return cnt + ((int64_t)id * kCntLanes + (int64_t)(blockIdx.x % kCntLanes)) * kCntStride;
}

// ---------------------------------------------------------------------------
// mesh preparation
// ---------------------------------------------------------------------------
__global__ void k_points(int64_t np, const double *pts, double4 *X) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  X[p] = make_double4(pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], 0.0);
}

// face centre = mean of the points (Section 2.2.1); S = sum 1/2 (p_i - c) x (p_i+1 - c)
__global__ void k_face_geom(DMesh m, double4 *S, double4 *C) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= m.nf) return;
  int b = m.foff[f], n = m.foff[f + 1] - b;
  v3 c = mk3(0, 0, 0);
  for (int i = 0; i < n; ++i) c = c + xyz(m.X[m.fpts[b + i]]);
  c = (1.0 / n) * c;
  v3 s = mk3(0, 0, 0);
  for (int i = 0; i < n; ++i) {
    v3 a = xyz(m.X[m.fpts[b + i]]) - c;
    v3 q = xyz(m.X[m.fpts[b + (i + 1 == n ? 0 : i + 1)]]) - c;
    s = s + cross(a, q);
  }
  s = 0.5 * s;
  C[f] = make_double4(c.x, c.y, c.z, 0.0);
  S[f] = make_double4(s.x, s.y, s.z, sqrt(dot(s, s)));
}

// Cell volume and centroid from tetrahedra (apex, c_f, p_i, p_i+1) over the
// outward face fans; the apex is the mean of the face centres.  Also the cell
// bounding box.
__global__ void k_cell_geom(DMesh m, double *V, double4 *XC, double4 *bblo, double4 *bbhi) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= m.nc) return;
  int k0 = m.cf_off[c], k1 = m.cf_off[c + 1];
  v3 a = mk3(0, 0, 0);
  for (int k = k0; k < k1; ++k) {
    int sf = m.cf[k];
    a = a + xyz(m.C[sf >= 0 ? sf : ~sf]);
  }
  a = (1.0 / (k1 - k0)) * a;
  double v6 = 0.0;
  v3 mom = mk3(0, 0, 0);
  v3 lo = mk3(1e300, 1e300, 1e300), hi = mk3(-1e300, -1e300, -1e300);
  for (int k = k0; k < k1; ++k) {
    int sf = m.cf[k];
    int f = sf >= 0 ? sf : ~sf;
    double sg = sf >= 0 ? 1.0 : -1.0;
    v3 cf = xyz(m.C[f]) - a;
    int b = m.foff[f], n = m.foff[f + 1] - b;
    for (int i = 0; i < n; ++i) {
      v3 pg = xyz(m.X[m.fpts[b + i]]);
      lo = mk3(dmin(lo.x, pg.x), dmin(lo.y, pg.y), dmin(lo.z, pg.z));
      hi = mk3(dmax(hi.x, pg.x), dmax(hi.y, pg.y), dmax(hi.z, pg.z));
      v3 p = pg - a;
      v3 q = xyz(m.X[m.fpts[b + (i + 1 == n ? 0 : i + 1)]]) - a;
      double t = sg * det3(cf, p, q);
      v6 += t;
      mom = mom + (0.25 * t) * (cf + p + q);
    }
  }
  V[c] = v6 / 6.0;
  v3 xc = a + (1.0 / v6) * mom;
  XC[c] = make_double4(xc.x, xc.y, xc.z, 0.0);
  bblo[c] = make_double4(lo.x, lo.y, lo.z, 0.0);
  bbhi[c] = make_double4(hi.x, hi.y, hi.z, 0.0);
}

// cell face planes: outward unit normal sgn * S/|S| and offset through c_f;
// the two cells of a face get exactly opposite planes.  A plane equal (bit
// for bit) to one the cell has already is not repeated: the coplanar faces a
// coarse cell shares with refined neighbours are one plane of the cell.
__global__ void k_cell_planes(DMesh m, double4 *cpl, uint8_t *npl, uint8_t *isbox,
                              uint8_t *fan_w, const double4 *bblo, const double4 *bbhi) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= m.nc) return;
  const int k0 = m.cf_off[c];
  int cnt = 0;
  for (int k = k0; k < m.cf_off[c + 1]; ++k) {
    int sf = m.cf[k];
    int f = sf >= 0 ? sf : ~sf;
    double4 S = m.S[f];
    v3 n = (1.0 / S.w) * xyz(S);
    double d = dot(n, xyz(m.C[f]));
    double sg = sf >= 0 ? 1.0 : -1.0;
    const double4 pl = make_double4(sg * n.x, sg * n.y, sg * n.z, sg * d);
    bool dup = false;
    for (int q = 0; q < cnt; ++q) {
      const double4 o = cpl[k0 + q];
      dup |= o.x == pl.x && o.y == pl.y && o.z == pl.z && o.w == pl.w;
    }
    if (!dup) cpl[k0 + cnt++] = pl;
  }
  npl[c] = (uint8_t)cnt;
  // a box cell: its six planes are +-e_x, +-e_y, +-e_z through its bounds
  const double4 lo = bblo[c], hi = bbhi[c];
  const double blo[3] = {lo.x, lo.y, lo.z}, bhi[3] = {hi.x, hi.y, hi.z};
  int sides = 0;
  for (int q = 0; q < cnt; ++q) {
    const double4 pl = cpl[k0 + q];
    const double n[3] = {pl.x, pl.y, pl.z};
    for (int a = 0; a < 3; ++a) {
      const bool axis = n[a] != 0.0 && n[(a + 1) % 3] == 0.0 && n[(a + 2) % 3] == 0.0;
      if (axis && n[a] == 1.0 && pl.w == bhi[a]) sides |= 1 << (2 * a);
      if (axis && n[a] == -1.0 && pl.w == -blo[a]) sides |= 2 << (2 * a);
    }
  }
  isbox[c] = cnt == 6 && sides == 63;
  int slots = 0;  // face-fan tetrahedra of the cell: one per face point
  for (int k = k0; k < m.cf_off[c + 1]; ++k) {
    const int sf = m.cf[k];
    const int f = sf >= 0 ? sf : ~sf;
    slots += m.foff[f + 1] - m.foff[f];
  }
  const int nfc = m.cf_off[c + 1] - k0;
  fan_w[c] = nfc <= 16 && slots <= 32 ? 16 : (nfc <= 32 && slots <= 64 ? 32 : 64);
}

// inverse distance weights of the point-cells (eq. 2.7)
__global__ void k_idw(DMesh m, double *w) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= m.np) return;
  v3 x = xyz(m.X[p]);
  double sum = 0.0;
  int k0 = m.pc_off[p], k1 = m.pc_off[p + 1];
  for (int k = k0; k < k1; ++k) {
    v3 r = x - xyz(m.XC[m.pc[k]]);
    double wk = 1.0 / sqrt(dot(r, r));
    w[k] = wk;
    sum += wk;
  }
  for (int k = k0; k < k1; ++k) w[k] /= sum;
}

__global__ void k_check_orientation(DMesh m, uint32_t *flags) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= m.ni) return;
  v3 d = xyz(m.XC[m.nei[f]]) - xyz(m.XC[m.own[f]]);
  if (!(dot(d, xyz(m.S[f])) > 0.0)) flag(flags, kFlagBadOrientation);
}

// U_p = sum_c w_pc U_c (eqs. 2.6-2.7 applied to the velocity, Section 2.3)
// IDW point velocity (eq. 2.6); also the per-point record (position,
// velocity) that the flux kernels gather with one cache line per point.
__global__ void k_point_velocity(DMesh m, const double *U0c, double4 *U, double *XU) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= m.np) return;
  v3 u = mk3(0, 0, 0);
  for (int k = m.pc_off[p]; k < m.pc_off[p + 1]; ++k) {
    int64_t c = m.pc[k];
    u = u + m.wpc[k] * mk3(U0c[3 * c], U0c[3 * c + 1], U0c[3 * c + 2]);
  }
  U[p] = make_double4(u.x, u.y, u.z, 0.0);
  const double4 x = m.X[p];
  double2 *r = reinterpret_cast<double2 *>(XU + 6 * p);
  r[0] = make_double2(x.x, x.y);
  r[1] = make_double2(x.z, u.x);
  r[2] = make_double2(u.y, u.z);
}

// ---------------------------------------------------------------------------
// step 4: classes, point values, planes
// ---------------------------------------------------------------------------
__global__ void k_reset(DState s) {
  if (threadIdx.x < kWNum) s.work[threadIdx.x] = 0;
}

// kClassCells cells per thread, strided by the grid (coalesced), and the
// thread's interface cells appended together: one atomic per block of
// kBlock * kClassCells cells on the list's counter.
constexpr int kClassCells = 8;
// Block vb of a grid of vg blocks over the cells of one mesh.
__device__ __forceinline__ void cell_class_blk(const DMesh &m, const DState &s, const DParams &p,
                                               int64_t vb, int64_t vg) {
  const int64_t stride = vg * blockDim.x;
  const int64_t c0 = vb * (int64_t)blockDim.x + threadIdx.x;
  unsigned im = 0;  // bit i: cell c0 + i stride is an interface cell
#pragma unroll
  for (int i = 0; i < kClassCells; ++i) {
    const int64_t c = c0 + i * stride;
    if (c < m.nc) {
      const double a = s.alpha[c];
      const int8_t cl = a <= p.eps ? 0 : (a >= 1.0 - p.eps ? 2 : 1);
      s.cls[c] = cl;
      if (p.band) s.inexact[c] = cl != 1 && a != 0.0 && a != 1.0;
      im |= (cl == 1 ? 1u : 0u) << i;
    }
  }
  const int pos = block_append_n(&s.work[kWInterface], __builtin_popcount(im));
#pragma unroll
  for (int i = 0; i < kClassCells; ++i)
    if ((im >> i) & 1u)
      s.icells[pos + __builtin_popcount(im & ((1u << i) - 1u))] = (int32_t)(c0 + i * stride);
}
__global__ __launch_bounds__(kBlock) void k_cell_class(DMesh m, DState s, DParams p) {
  cell_class_blk(m, s, p, blockIdx.x, gridDim.x);
}

// Point mask: bit 1 empty, 2 full, 4 interface among the point-cells; with
// the narrow band also bit 8, an empty or full point-cell whose alpha is not
// exactly 0 or 1, so that mask 1 (2) means every point-cell is exactly 0 (1).
__device__ __forceinline__ void point_prep_one(const DMesh &m, const DState &s, const DParams &pr,
                                               int64_t p) {
  if (p >= m.np) return;
  int k0 = m.pc_off[p], k1 = m.pc_off[p + 1];
  uint8_t mask = 0;
  // unrolled so that the cell ids, then the class bytes, load together
  if (pr.band) {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) {
      const int c = m.pc[k];
      int8_t cl = s.cls[c];
      mask |= (cl == 0 ? 1 : (cl == 2 ? 2 : 4)) | (s.inexact[c] ? 8 : 0);
    }
  } else {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) {
      int8_t cl = s.cls[m.pc[k]];
      mask |= cl == 0 ? 1 : (cl == 2 ? 2 : 4);
    }
  }
  s.pmask[p] = mask;
  if (mask & 4) {
    double a = 0.0;
    for (int k = k0; k < k1; ++k) a += m.wpc[k] * s.alpha[m.pc[k]];
    s.alpha_p[p] = a;
  }
}
__global__ __launch_bounds__(kBlock) void k_point_prep(DMesh m, DState s, DParams pr) {
  point_prep_one(m, s, pr, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// Wave-wide reductions.  Every lane receives the same value: at each level of
// the butterfly partner lanes add the same two operands in swapped order,
// and floating-point addition is commutative.
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = dmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = dmax(v, __shfl_xor(v, o));
  return v;
}

// One tetrahedron (o, c_f, p_i, p_i+1) of the outward face fans of a cell,
// relative to the cell centroid o, with its signed volume times six; empty
// (v6 = 0) for a slot beyond the cell's fan.
struct FanTet {
  v3 cf, pa, pb;
  double v6;
};

// The cell's faces are spread over the W lanes of its group (lane j < nfc
// holds face j: its index f, sign, first point b and point count nn); the fan
// slots are numbered face by face, so slot s belongs to the last face whose
// first slot (an exclusive prefix sum of nn over the lanes) is at most s.
template <int W>
__device__ FanTet fan_tet(const DMesh &m, v3 o, int slot, int nfc, int f, double sg, int b,
                          int nn, int first, int total) {
  int j = 0;
  for (int q = 1; q < nfc; ++q)
    if (__shfl(first, q, W) <= slot) j = q;
  const int fj = __shfl(f, j, W), bj = __shfl(b, j, W), nj = __shfl(nn, j, W);
  const double sj = __shfl(sg, j, W);
  const int i = slot - __shfl(first, j, W);
  FanTet t{mk3(0, 0, 0), mk3(0, 0, 0), mk3(0, 0, 0), 0.0};
  if (slot < total) {
    const int i1 = (i + 1 == nj) ? 0 : i + 1;
    t.cf = xyz(m.C[fj]) - o;
    t.pa = xyz(m.X[m.fpts[bj + i]]) - o;
    t.pb = xyz(m.X[m.fpts[bj + i1]]) - o;
    t.v6 = sj * det3(t.cf, t.pa, t.pb);
  }
  return t;
}

// Sums, minima and maxima over a group of W lanes (W = 32 or 64), the same
// value in every lane of the group (butterfly within the group).
template <int W>
__device__ __forceinline__ double group_sum(double v) {
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W>
__device__ __forceinline__ double group_min(double v) {
  for (int o = W / 2; o > 0; o >>= 1) v = dmin(v, __shfl_xor(v, o, W));
  return v;
}
template <int W>
__device__ __forceinline__ double group_max(double v) {
  for (int o = W / 2; o > 0; o >>= 1) v = dmax(v, __shfl_xor(v, o, W));
  return v;
}

// NAG gradient (eqs. 2.8-2.12) and plane positioning (Section 2.2.2) of one
// interface cell by a group of W lanes (16, 32 or 64).  The fill level
// g(s) = |C ∩ {n.x <= s}| / |C| - alpha is monotone between the lowest and
// highest cell points; it is solved by regula falsi with the Illinois
// modification, which keeps a bracket and converges superlinearly, from the
// cell's previous plane as the first iterate.  Each evaluation sums vol6 *
// kept fraction over the fan tetrahedra of the cell, two per lane, so every
// decision of the iteration is uniform over the group.
// Plane of interface cell c by a group of W lanes (lane: the index in the
// group): NAG (or least-squares) gradient, normal, and positioning.
template <int W>
__device__ __forceinline__ void plane_cell(const DMesh &m, const DState &s, const DParams &p,
                                           int64_t c, int lane, unsigned long long &nfall) {
    const double a = s.alpha[c];
    const int k0 = m.cf_off[c], nfc = m.cf_off[c + 1] - k0;
    const double Vc = m.V[c];
    // face lane of the cell: lanes j < nfc hold face j
    int lf = 0, lb = 0, lnn = 0;
    double lsg = 0.0;
    if (lane < nfc) {
      const int sf = m.cf[k0 + lane];
      lf = sf >= 0 ? sf : ~sf;
      lsg = sf >= 0 ? 1.0 : -1.0;
      lb = m.foff[lf];
      lnn = m.foff[lf + 1] - lb;
    }
    v3 g;
    if (p.gradient == 1) {
      // generalized least squares (Section 2.2.1): lanes over the cells that
      // share a point with c; (sum w^2 d d^T) g = sum w^2 d (alpha_k - alpha_c)
      // with d = x_k - x_c, w = 1/|d|, solved by Cramer's rule
      const v3 xc = xyz(m.XC[c]);
      double a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0, b0 = 0, b1 = 0, b2 = 0;
      for (int e = m.cpn_off[c] + lane; e < m.cpn_off[c + 1]; e += W) {
        const int k = m.cpn[e];
        const v3 d = xyz(m.XC[k]) - xc;
        const double w2 = 1.0 / dot(d, d);
        const double da = s.alpha[k] - a;
        a00 += w2 * d.x * d.x; a01 += w2 * d.x * d.y; a02 += w2 * d.x * d.z;
        a11 += w2 * d.y * d.y; a12 += w2 * d.y * d.z; a22 += w2 * d.z * d.z;
        b0 += w2 * d.x * da; b1 += w2 * d.y * da; b2 += w2 * d.z * da;
      }
      a00 = group_sum<W>(a00); a01 = group_sum<W>(a01); a02 = group_sum<W>(a02);
      a11 = group_sum<W>(a11); a12 = group_sum<W>(a12); a22 = group_sum<W>(a22);
      b0 = group_sum<W>(b0); b1 = group_sum<W>(b1); b2 = group_sum<W>(b2);
      const double det = det3(mk3(a00, a01, a02), mk3(a01, a11, a12), mk3(a02, a12, a22));
      const double d0 = det3(mk3(b0, b1, b2), mk3(a01, a11, a12), mk3(a02, a12, a22));
      const double d1 = det3(mk3(a00, a01, a02), mk3(b0, b1, b2), mk3(a02, a12, a22));
      const double d2 = det3(mk3(a00, a01, a02), mk3(a01, a11, a12), mk3(b0, b1, b2));
      g = det != 0.0 ? mk3(d0 / det, d1 / det, d2 / det) : mk3(0, 0, 0);
    } else {
      // NAG: lanes over the faces of the cell
      v3 gl = mk3(0, 0, 0);
      if (lane < nfc) {
        const int f = lf, b = lb, nn = lnn;
        const double sg = lsg;
        double fp = 0.0;
        for (int j = 0; j < nn; ++j) fp += s.alpha_p[m.fpts[b + j]];
        fp /= nn;
        v3 cf = xyz(m.C[f]);
        double num = 0.0, den = 0.0;
        int qa = m.fpts[b];
        for (int j = 0; j < nn; ++j) {
          int qb = m.fpts[b + ((j + 1 == nn) ? 0 : j + 1)];
          v3 t = cross(xyz(m.X[qa]) - cf, xyz(m.X[qb]) - cf);
          double A = 0.5 * sqrt(dot(t, t));
          num += A * (fp + s.alpha_p[qa] + s.alpha_p[qb]) / 3.0;
          den += A;
          qa = qb;
        }
        gl = (sg * (num / den)) * xyz(m.S[f]);
      }
      g = (1.0 / Vc) * mk3(group_sum<W>(gl.x), group_sum<W>(gl.y), group_sum<W>(gl.z));
    }
    double gn = sqrt(dot(g, g));
    if (!(gn * cbrt(Vc) >= p.grad_zero)) {
      if (lane == 0) {
        s.cls[c] = 3;
        s.plane[c] = make_double4(0.0, 0.0, 0.0, 0.0);
        ++nfall;
      }
      return;
    }
    const v3 n = (-1.0 / gn) * g;
    const v3 o = xyz(m.XC[c]);
    // fan tetrahedra as heights along n
    int first = lnn;  // inclusive prefix sum of the point counts, then exclusive
    for (int q = 1; q < W; q <<= 1) {
      const int t = __shfl_up(first, q, W);
      if (lane >= q) first += t;
    }
    const int total = __shfl(first, W - 1, W);
    first -= lnn;
    FanTet t0 = fan_tet<W>(m, o, lane, nfc, lf, lsg, lb, lnn, first, total);
    FanTet t1 = fan_tet<W>(m, o, lane + W, nfc, lf, lsg, lb, lnn, first, total);
    const double hc0 = dot(n, t0.cf), ha0 = dot(n, t0.pa), hb0 = dot(n, t0.pb);
    const double hc1 = dot(n, t1.cf), ha1 = dot(n, t1.pa), hb1 = dot(n, t1.pb);
    // the points of the cell are the p_i of its fans
    double hmin = t0.v6 != 0.0 ? ha0 : 1e300, hmax = t0.v6 != 0.0 ? ha0 : -1e300;
    if (t1.v6 != 0.0) { hmin = dmin(hmin, ha1); hmax = dmax(hmax, ha1); }
    hmin = group_min<W>(hmin);
    hmax = group_max<W>(hmax);
    const double tot6 = group_sum<W>(t0.v6 + t1.v6);
    double lo = hmin, glo = -a, hi = hmax, ghi = 1.0 - a;
    double sx = 0.5 * (lo + hi);
    int side = 0;
    // The cell's plane of the previous step (zero after alpha is set, and
    // stale for a cell that was not an interface cell then): its point
    // nearest the centroid, relative to the centroid, is the first iterate
    // when it lies inside the bracket.
    {
      const double4 prev = s.plane[c];
      const v3 no = xyz4(prev);
      const double sg = (prev.w - dot(no, o)) * dot(n, no);
      if (sg > lo && sg < hi) {
        const double f0 = t0.v6 * tet_kept_fraction(D4{sg, sg - hc0, sg - ha0, sg - hb0});
        const double f1 = t1.v6 * tet_kept_fraction(D4{sg, sg - hc1, sg - ha1, sg - hb1});
        const double gs = group_sum<W>(f0 + f1) / tot6 - a;
        sx = sg;
        if (fabs(gs) <= p.pos_tol) {
          if (lane == 0) s.plane[c] = make_double4(n.x, n.y, n.z, sx + dot(n, o));
          return;
        }
        if (gs < 0.0) { lo = sg; glo = gs; side = -1; }
        else { hi = sg; ghi = gs; side = 1; }
      }
    }
    for (int it = 0; it < p.pos_max_iter; ++it) {
      double sn = hi - ghi * (hi - lo) / (ghi - glo);
      if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
      double f0 = t0.v6 * tet_kept_fraction(D4{sn, sn - hc0, sn - ha0, sn - hb0});
      double f1 = t1.v6 * tet_kept_fraction(D4{sn, sn - hc1, sn - ha1, sn - hb1});
      double gs = group_sum<W>(f0 + f1) / tot6 - a;
      sx = sn;
      if (fabs(gs) <= p.pos_tol) break;
      if (gs < 0.0) {
        lo = sn; glo = gs;
        if (side == -1) ghi *= 0.5;
        side = -1;
      } else {
        hi = sn; ghi = gs;
        if (side == 1) glo *= 0.5;
        side = 1;
      }
      if (hi - lo <= 2e-16 * (hmax - hmin)) break;
    }
    if (lane == 0) s.plane[c] = make_double4(n.x, n.y, n.z, sx + dot(n, o));
}

// NAG gradient and plane positioning of the interface cells, four cells of
// the list per wave.  A cell is always evaluated by the same group width --
// the 16, 32 or 64 lanes its size admits (fan_w) -- whatever cells share its
// wave: the lanes' partial sums, and so the rounding of the group sums,
// depend on the width, and the list's order is not fixed.  The wave takes
// its 16-lane cells side by side, then its 32-lane cells two at a time, then
// its whole-wave cells one after the other.
// The cells i = 4q .. 4q + 3 of the list (of `count`).  WIDE: the mesh has
// whole-wave cells (without, their pass is left out of the kernel, which then
// fits its registers).
template <bool WIDE>
__device__ __forceinline__ void plane_quad(const DMesh &m, const DState &s, const DParams &p,
                                           int q, int count, int lane,
                                           unsigned long long &nfall) {
  // cell j of the four and its group width (0 past the list), read again in
  // every pass so that nothing stays live across the cell evaluations
  auto cell_at = [&](int j, int &w) -> int64_t {
    const int i = 4 * q + j;
    const int64_t c = i < count ? (int64_t)s.icells[i] : -1;
    w = c >= 0 ? (int)m.fan_w[c] : 0;
    return c;
  };
  // 16-lane cells: the r-th of them takes lanes 16 r .. 16 r + 15
  {
    int64_t c16 = -1;
    int r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int w;
      const int64_t c = cell_at(j, w);
      if (w == 16) {
        c16 = r == lane / 16 ? c : c16;
        ++r;
      }
    }
    if (c16 >= 0) plane_cell<16>(m, s, p, c16, lane & 15, nfall);
  }
  // 32-lane cells, two per pass: the k-th of them in lanes 32 (k % 2) ..
  for (int pass = 0; pass < 2; ++pass) {
    int64_t c32 = -1;
    int r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int w;
      const int64_t c = cell_at(j, w);
      if (w == 32) {
        c32 = r == 2 * pass + lane / 32 ? c : c32;
        ++r;
      }
    }
    if (r <= 2 * pass) break;
    if (c32 >= 0) plane_cell<32>(m, s, p, c32, lane & 31, nfall);
  }
  // whole-wave cells one after the other
  if constexpr (WIDE) {
    for (int j = 0; j < 4; ++j) {
      int w;
      const int64_t c = cell_at(j, w);
      if (w == 64) plane_cell<64>(m, s, p, c, lane, nfall);
    }
  }
}
template <bool WIDE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_plane(DMesh m, DState s, DParams p) {
  const int count = s.work[kWInterface];
  const int lane = lane_id();
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (int)((gridDim.x * blockDim.x) >> 6);
  unsigned long long nfall = 0;
  for (int q = wave; 4 * q < count; q += nwaves) plane_quad<WIDE>(m, s, p, q, count, lane, nfall);
  wave_count(cnt_at(s.cnt, kCntFallback), nfall);
}

// ---------------------------------------------------------------------------
// steps 1-3: flux polyhedra and their correction
// ---------------------------------------------------------------------------
// Signed volume of the flux polyhedron of a face with points r_i (relative to
// the face centre) swept by lam * d_i.  Its surface: the face fan, the swept
// fan about the mean of the swept points, and each side quad
// (p_i+1, p_i, q_i, q_i+1) as four triangles about its vertex mean.  Summing
// the tetrahedra with apex at the face centre in closed form:
//   side i = (1/6)[lam h_i.(s_i x e_i) + lam^2 h_i.(d_i x d_i+1)]
//   top    = -(1/6) lam dbar.(A2 + lam B + lam^2 C)
// with e_i = r_i+1 - r_i, h_i = (r_i + r_i+1)/2, s_i = d_i + d_i+1,
// A2 = sum r_i x r_i+1, B = sum (r_i x d_i+1 + d_i x r_i+1), C = sum d_i x d_i+1,
// dbar = mean d_i.  V(lam) = c1 lam + c2 lam^2 + c3 lam^3 exactly.
//
// Correction (Section 2.3): V(lam) = F dt on the branch of V through 0 on
// which V' keeps its sign (bounded by the real roots of V'), by Newton from
// lam = 1 safeguarded by bisection.  status 1 when the target lies beyond the
// extremum of V at the branch end: lam is then that end or the plain sweep
// (+-1 on the same side), whichever is nearer to 0.
__device__ __forceinline__ void correct(double c1, double c2, double c3, double T, double rtol,
                                        int maxit, double &lam, int &iters, int &status) {
  iters = 0;
  status = 0;
  lam = 0.0;
  if (T == 0.0) return;
  if (!(c1 != 0.0) || !isfinite(c2) || !isfinite(c3)) { status = 1; return; }
  // the branch ends at +-32 when V' has no root nearer to 0 (a corrected sweep
  // 32 times the plain one is far outside any Courant limit)
  const double big = 32.0;
  double lo = -big, hi = big;
  if (c3 != 0.0) {
    double disc = c2 * c2 - 3.0 * c1 * c3;
    if (disc > 0.0) {
      double q = -(c2 + copysign(sqrt(disc), c2));
      double r0 = q / (3.0 * c3), r1 = c1 / q;
      if (r0 > 0.0) hi = dmin(hi, r0); else if (r0 < 0.0) lo = dmax(lo, r0);
      if (r1 > 0.0) hi = dmin(hi, r1); else if (r1 < 0.0) lo = dmax(lo, r1);
    }
  } else if (c2 != 0.0) {
    double r = -c1 / (2.0 * c2);
    if (r > 0.0) hi = dmin(hi, r); else if (r < 0.0) lo = dmax(lo, r);
  }
  double end = ((T > 0.0) == (c1 > 0.0)) ? hi : lo;
  double gend = ((c3 * end + c2) * end + c1) * end - T;
  if (!(gend * T >= 0.0)) { lam = copysign(dmin(fabs(end), 1.0), end); status = 1; return; }
  double a = dmin(0.0, end), b = dmax(0.0, end);
  double ga = (a == 0.0) ? -T : gend;
  double x = 1.0;
  if (!(x > a && x < b)) x = 0.5 * (a + b);
  for (;;) {
    double g = ((c3 * x + c2) * x + c1) * x - T;
    if (fabs(g) <= rtol * fabs(T) || iters >= maxit) break;
    if ((g < 0.0) == (ga < 0.0)) { a = x; ga = g; } else { b = x; }
    double dv = (3.0 * c3 * x + 2.0 * c2) * x + c1;
    double xn = x - g / dv;
    if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
    ++iters;
    if (xn == x) break;
    x = xn;
  }
  lam = x;
}

// Point indices of face f from the padded list (-1 past the last point): one
// 16-byte load per four points.
// The flux kernel streams its per-face inputs and outputs with the
// non-temporal hint, so that they pass through L2 without displacing the
// point records that the next rows of faces share.
typedef int int4_nt __attribute__((ext_vector_type(4)));
template <int NMAX>
__device__ __forceinline__ void load_face_points(const DMesh &m, int64_t f, int (&q)[NMAX]) {
  if constexpr (NMAX <= 4) {
    const int4_nt v = __builtin_nontemporal_load(reinterpret_cast<const int4_nt *>(m.fpad + 4 * f));
    const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < NMAX; ++i) q[i] = w[i];
  } else {
    const int4 a = *reinterpret_cast<const int4 *>(m.fpad + 8 * f);
    const int4 b = *reinterpret_cast<const int4 *>(m.fpad + 8 * f + 4);
    const int w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < NMAX; ++i) q[i] = w[i];
  }
}

// per-block sums of up to three counters, one atomic each per block
__device__ __forceinline__ void block_count3(unsigned long long *d0, unsigned long long v0,
                                             unsigned long long *d1, unsigned long long v1,
                                             unsigned long long *d2, unsigned long long v2) {
  __shared__ unsigned long long red[3][kBlock / 64];
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  v2 = wave_sum(v2);
  const int w = threadIdx.x / 64;
  if (lane_id() == 0) { red[0][w] = v0; red[1][w] = v1; red[2][w] = v2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0, c = 0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) { a += red[0][i]; b += red[1][i]; c += red[2][i]; }
    if (a) atomicAdd(d0, a);
    if (b) atomicAdd(d1, b);
    if (c) atomicAdd(d2, c);
  }
}

// Coefficients of the volume cubic V(lam) = c1 lam + c2 lam^2 + c3 lam^3 of
// the flux polyhedron of a face with points q[0..n-1] (records in XU) and
// sweep factor `sweep`.  N > 0 fixes n = N at compile time; N = 0 takes n at
// run time (at most NMAX).
template <int NMAX, int N>
__device__ __forceinline__ void face_cubic(const double *XU, const int (&q)[NMAX], int n,
                                           double sweep, double &c1, double &c2, double &c3) {
  v3 r[NMAX], d[NMAX];
  v3 c = mk3(0, 0, 0), db = mk3(0, 0, 0);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (N > 0 || i < n) {
      const PointRec pr = point_rec(XU, q[i]);
      r[i] = pr.x;
      d[i] = sweep * pr.u;
      c = c + r[i];
      db = db + d[i];
    } else {
      r[i] = mk3(0, 0, 0);
      d[i] = mk3(0, 0, 0);
    }
  }
  const double inv = N > 0 ? 1.0 / N : 1.0 / n;
  c = inv * c;
  db = inv * db;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) r[i] = r[i] - c;
  // h_i.((d_i + d_i+1) x e_i) = -(d_i + d_i+1).(r_i x r_i+1) (triple product
  // with e_i = r_i+1 - r_i, h_i = (r_i + r_i+1) / 2), so every edge needs the
  // three products r_i x r_i+1, d_i x d_i+1 and r_i x d_i+1 + d_i x r_i+1,
  // taken against the mean sweep d-bar edge by edge:
  //   6 c1 = -sum (d_i + d_i+1 + d-bar).(r_i x r_i+1)
  //   6 c2 = sum [(r_i + r_i+1)/2 . (d_i x d_i+1) - d-bar.(r_i x d_i+1 + d_i x r_i+1)]
  //   6 c3 = -sum d-bar.(d_i x d_i+1)
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (N > 0 || i < n) {
      const v3 rn = N > 0 ? r[(i + 1) % NMAX] : ((i + 1 < n) ? r[(i + 1) % NMAX] : r[0]);
      const v3 dn = N > 0 ? d[(i + 1) % NMAX] : ((i + 1 < n) ? d[(i + 1) % NMAX] : d[0]);
      const v3 dd = cross(d[i], dn);
      t1 -= dot(d[i] + dn + db, cross(r[i], rn));
      t2 += 0.5 * dot(r[i] + rn, dd) - dot(db, cross(r[i], dn) + cross(d[i], rn));
      t3 -= dot(db, dd);
    }
  }
  const double sixth = 1.0 / 6.0;
  c1 = t1 * sixth;
  c2 = t2 * sixth;
  c3 = t3 * sixth;
}

// The volume cubic of every face for a unit sweep factor, once per velocity
// field: the swept vectors of a step are sweep * U_p with sweep = -s dt, so
// its cubic has the coefficients sweep C1, sweep^2 C2 and sweep^3 C3, and the
// flux kernel of each step needs neither the points nor their velocities.
template <int NMAX>
__global__ void k_face_coeffs(DMesh m, const double *XU, double *coef) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= m.nf) return;
  int q[NMAX];
  load_face_points<NMAX>(m, f, q);
  int n = 0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) n += q[i] >= 0;
  double c1, c2, c3;
  if (n == NMAX) face_cubic<NMAX, NMAX>(XU, q, n, 1.0, c1, c2, c3);
  else face_cubic<NMAX, 0>(XU, q, n, 1.0, c1, c2, c3);
  coef[f] = c1;
  coef[m.nf + f] = c2;
  coef[2 * m.nf + f] = c3;
}

// Faces of up to four points run at four waves per SIMD (at most 128 VGPRs:
// the loads of a face are a chain of two dependent gathers, hidden by the
// other waves); faces of up to eight points need more registers.
// The faces base .. base + blockDim.x - 1 of one mesh, one per thread.
template <int NMAX>
__device__ __forceinline__ void flux_chunk(const DMesh &m, const DState &s, const DParams &p,
                                           int64_t base, double dt, double sc,
                                           unsigned long long &nflux, unsigned long long &nit,
                                           unsigned long long &nbad) {
    const int64_t f = base + threadIdx.x;
    bool geo = false;
    int nq = 0;  // points of the face (counted where faces may be large)
    if (f < m.nf) {
      // the point list and the flux are independent loads, issued together
      int q[NMAX];
      load_face_points<NMAX>(m, f, q);
      if constexpr (NMAX > kSmallFace) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i) nq += q[i] >= 0;
      }
      double F = sc * __builtin_nontemporal_load(&s.F0[f]);
      double T = F * dt;
      double lam = 0.0, vph = 0.0;
      int it = 0, stat = 0;
      uint8_t kind = 0, mask = 0;
      if (F != 0.0) {
        // the step's cubic from the face's unit-sweep coefficients
        const double sweep = -sc * dt, sw2 = sweep * sweep;
        const double c1 = sweep * __builtin_nontemporal_load(&s.coef[f]);
        const double c2 = sw2 * __builtin_nontemporal_load(&s.coef[m.nf + f]);
        const double c3 = sw2 * sweep * __builtin_nontemporal_load(&s.coef[2 * m.nf + f]);
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
          if (q[i] >= 0) mask |= s.pmask[q[i]];
        correct(c1, c2, c3, T, p.corr_rtol, p.corr_max_iter, lam, it, stat);
        const double vl = stat ? ((c3 * lam + c2) * lam + c1) * lam : T;
        nflux += 1;
        nit += (unsigned long long)it;
        nbad += (unsigned long long)stat;
        if ((mask & 6) == 0) {
          kind = 1;
          vph = 0.0;
        } else if ((mask & 7) == 2 && f < m.ni) {
          kind = 2;
          vph = T;
        } else if (stat && !(fabs(vl) >= 0.25 * fabs(T) && vl * T > 0.0)) {
          // no swept polyhedron on the branch meets F dt and the clamped one
          // is under a quarter of it: the face carries the upwind (donor)
          // cell's fraction of F dt (outside is empty)
          const int64_t donor = T > 0.0 ? (int64_t)m.own[f] : (f < m.ni ? (int64_t)m.nei[f] : -1);
          kind = 4;
          vph = donor >= 0 ? s.alpha[donor] * T : 0.0;
        } else {
          // a clamped polyhedron of at least a quarter of F dt: its phase
          // fraction times F dt (the scale at most 4)
          if (stat) s.vscale[f] = T / vl;
          kind = 3;
          geo = true;
        }
      }
      if (p.band) {
        // narrow band: whether every point-cell of every face point is exactly
        // 0 (1), also for faces without flux
        if (F == 0.0) {
#pragma unroll
          for (int i = 0; i < NMAX; ++i)
            if (q[i] >= 0) mask |= s.pmask[q[i]];
        }
        s.fbulk[f] = mask == 1 ? 1 : (mask == 2 ? 2 : 0);
      }
      __builtin_nontemporal_store(lam, &s.lam[f]);
      if (!geo) __builtin_nontemporal_store(vph, &s.vphase[f]);
      __builtin_nontemporal_store((uint8_t)(it > 255 ? 255 : it), &s.iters[f]);
      __builtin_nontemporal_store(kind, &s.kind[f]);
      __builtin_nontemporal_store((uint8_t)stat, &s.fstatus[f]);
    }
    bool large = false;
    if constexpr (NMAX > kSmallFace) {
      large = geo && nq > kSmallFace;
      const int sl = wave_append(&s.work[kWGeoLarge], large);
      if (large) s.gfaces[m.nf - 1 - sl] = (int32_t)f;
    }
    int slot = wave_append(&s.work[kWGeometric], geo && !large);
    if (geo && !large) s.gfaces[slot] = (int32_t)f;
}

template <int NMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NMAX <= 4 ? 4 : 1)))
void k_flux(DMesh m, DState s, DParams p) {
  const int step = *s.stepno;
  const double dt = s.dt[step], sc = s.sc[step];
  // every XCD walks one contiguous range of the face blocks with its blocks
  // side by side (a grid of about the resident blocks moves as one front),
  // so a point record fetched for one row of cells is still in that XCD's L2
  // when the faces of the next row need it
  const int64_t nb = (m.nf + blockDim.x - 1) / blockDim.x;
  const int per = (int)gridDim.x / kXcds;
  const int x = (int)blockIdx.x % kXcds, j = (int)blockIdx.x / kXcds;
  const int64_t b1 = nb * (x + 1) / kXcds;
  unsigned long long nflux = 0, nit = 0, nbad = 0;
  for (int64_t b = nb * x / kXcds + j; b < b1; b += per)
    flux_chunk<NMAX>(m, s, p, b * blockDim.x, dt, sc, nflux, nit, nbad);
  block_count3(cnt_at(s.cnt, kCntFaceFluxes), nflux, cnt_at(s.cnt, kCntIters), nit, cnt_at(s.cnt, kCntUnreached), nbad);
}

// ---------------------------------------------------------------------------
// step 5: phase volume of the geometric faces
// ---------------------------------------------------------------------------
// Work item (slot, k): tetrahedron k of the flux polyhedron of face
// gfaces[slot] at its corrected lam, apex at the face centre (local origin):
//   k = 5 i      top    (c_q, q_i+1, q_i)
//   k = 5 i + 1  side   (m_i, p_i+1, p_i)
//   k = 5 i + 2         (m_i, p_i, q_i)
//   k = 5 i + 3         (m_i, q_i, q_i+1)
//   k = 5 i + 4         (m_i, q_i+1, p_i+1)
// The signed tet volume times sum over stencil cells of
// |T ∩ C_c ∩ H_c| (H = the PLIC half-space in interface cells, all space in
// full cells, alpha-weighted in vanishing-gradient cells) is stored per item.

// pair_regs for a box cell: its cutting planes in mask order, then the PLIC
// plane of an interface cell.
__device__ __forceinline__ void pair_regs_box(const double *bb, const DState &s, v3 c, int cell,
                                              int cl, uint32_t mask, Pl &p0, Pl &p1, Pl &p2,
                                              Pl &p3) {
  const Pl pl = cl == 1 ? plic_plane_at(s, cell, c) : Pl{0, 0, 0, 0};
  uint32_t mm = mask;
  p0 = mm ? box_plane(bb, __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p1 = mm ? box_plane(bb, __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p2 = mm ? box_plane(bb, __builtin_ctz(mm), c) : pl;
  mm &= mm - 1;
  p3 = mm ? box_plane(bb, __builtin_ctz(mm), c) : pl;
}

// Tetrahedron k of a face staged in LDS (P[j]: point j minus the face centre,
// then its sweep at the corrected lam; cq: the mean sweep; n points), built
// exactly as flux_tet builds it from global memory.
__device__ __forceinline__ bool staged_tet(const double (*P)[6], int n, const double *cq, int k,
                                           v3 &t1, v3 &t2, v3 &t3, double &det, double &sgn) {
  if (k >= 5 * n) return false;
  const int i = k / 5, type = k - 5 * i;
  const int i1 = (i + 1 == n) ? 0 : i + 1;
  const v3 pi = mk3(P[i][0], P[i][1], P[i][2]), pj = mk3(P[i1][0], P[i1][1], P[i1][2]);
  const v3 qi = pi + mk3(P[i][3], P[i][4], P[i][5]);
  const v3 qj = pj + mk3(P[i1][3], P[i1][4], P[i1][5]);
  if (type == 0) { t1 = mk3(cq[0], cq[1], cq[2]); t2 = qj; t3 = qi; }
  else {
    t1 = 0.25 * (pi + pj + qi + qj);
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

// A queued pair of the register clip: the tet (from its lane's LDS row), its
// six-fold volume, the cell, its class and its planes in mask order (then
// the PLIC plane of an interface cell).
// The candidate's class comes from LDS, and so does its first plane index
// when the kernel stages it (ccq0, cells that are not boxes), so the plane
// loads do not wait on other loads.
__device__ __forceinline__ void queued_pair(const DMesh &m, const DState &s, const uint32_t *qpair,
                                            const double (*tv)[kFastBlock],
                                            const double (*fc)[3], const int32_t *ccell,
                                            const int8_t *ccls, const int32_t *ccq0,
                                            const double (*cbox)[6], int tpf, int kc, int item,
                                            Tet &T, double &det, int &cell, int &cl, Pl &p0,
                                            Pl &p1, Pl &p2, Pl &p3) {
  const int l = item % kFastBlock;
  const uint32_t qp = qpair[item];
  const int lf = l / tpf;
  const int u = lf * kc + (int)((qp >> 16) & 63u);
  cell = ccell[u];
  const v3 c = mk3(fc[lf][0], fc[lf][1], fc[lf][2]);
  T = Tet{mk3(0, 0, 0), mk3(tv[0][l], tv[1][l], tv[2][l]), mk3(tv[3][l], tv[4][l], tv[5][l]),
          mk3(tv[6][l], tv[7][l], tv[8][l])};
  det = tv[9][l];
  cl = ccls[u] & 7;
  if (qp & (1u << 22))
    pair_regs_box(cbox[u], s, c, cell, cl, qp & 0xffffu, p0, p1, p2, p3);
  else
    pair_regs_q(m, s, c, cell, cl, ccq0 ? ccq0[u] : m.cf_off[cell], qp & 0xffffu, p0, p1, p2,
                p3);
}

// A phase-B bin of pairs of K planes, three lanes per pair (one per term of
// the first plane's split; 21 pairs per pass).  The bin's items are bin[t],
// or bin[cap - 1 - t] for a bin filled from the end.
template <int K>
__device__ __forceinline__ void three_lane_bin(const DMesh &m, const DState &s,
                                               const uint32_t *qpair,
                                               const double (*tv)[kFastBlock],
                                               const double (*fc)[3], const int32_t *ccell,
                                               const int8_t *ccls, const int32_t *ccq0,
                                               const double (*cbox)[6], int tpf, int kc,
                                               const uint16_t *bin, int cnt, bool from_end,
                                               int cap, double *res) {
  const int lane = threadIdx.x;
  for (int t0 = 0; t0 < cnt; t0 += kFastBlock / 3) {
    const int t = t0 + lane / 3, term = lane - 3 * (lane / 3);
    const bool on = lane < (kFastBlock / 3) * 3 && t < cnt;
    int item = 0;
    double val = 0.0, w = 0.0, det = 0.0;
    if (on) {
      item = bin[from_end ? cap - 1 - t : t];
      Tet T;
      int cell, cl;
      Pl p0, p1, p2, p3;
      queued_pair(m, s, qpair, tv, fc, ccell, ccls, ccq0, cbox, tpf, kc, item, T, det, cell, cl,
                  p0, p1, p2, p3);
      val = split_term<K>(dist_table<K>(T, p0, p1, p2, p3), term);
      w = class_weight(s, cell, cl);
    }
    const double v1 = __shfl_down(val, 1), v2 = __shfl_down(val, 2);
    if (on && term == 0) res[item] = w * (det * ((val + v1) + v2));
  }
}

// A phase-B bin of pairs of K planes, one lane per pair (64 pairs per pass):
// the whole recursion of the closed form in the pair's lane.
template <int K>
__device__ __forceinline__ void one_lane_bin(const DMesh &m, const DState &s,
                                             const uint32_t *qpair,
                                             const double (*tv)[kFastBlock],
                                             const double (*fc)[3], const int32_t *ccell,
                                             const int8_t *ccls, const int32_t *ccq0,
                                             const double (*cbox)[6], int tpf, int kc,
                                             const uint16_t *bin, int cnt, bool from_end, int cap,
                                             double *res) {
  for (int t = (int)threadIdx.x; t < cnt; t += kFastBlock) {
    const int item = bin[from_end ? cap - 1 - t : t];
    Tet T;
    int cell, cl;
    double det;
    Pl p0, p1, p2, p3;
    queued_pair(m, s, qpair, tv, fc, ccell, ccls, ccq0, cbox, tpf, kc, item, T, det, cell, cl, p0,
                p1, p2, p3);
    const double v = kept_fraction<K>(dist_table<K>(T, p0, p1, p2, p3));
    res[item] = class_weight(s, cell, cl) * (det * v);
  }
}

// A phase-B bin of pairs of five planes of cells that are not boxes, nine
// lanes per pair (term j of piece i of the first two planes' splits; seven
// pairs per pass), filled from the end of bin (capacity cap).  The terms are
// combined as the recursion adds them: the three of a piece, then the pieces
// weighted by their ratios.
__device__ __forceinline__ void nine_lane_bin(const DMesh &m, const DState &s,
                                              const uint32_t *qpair,
                                              const double (*tv)[kFastBlock],
                                              const double (*fc)[3], const int32_t *ccell,
                                              const int8_t *ccls, const int32_t *ccq0,
                                              int tpf, int kc, const uint16_t *bin, int cnt,
                                              int cap, double *res) {
  const int lane = threadIdx.x;
  for (int t0 = 0; t0 < cnt; t0 += kFastBlock / 9) {
    const int t = t0 + lane / 9, sub = lane - 9 * (lane / 9);
    const int i = sub / 3, j = sub - 3 * i;
    const bool on = lane < (kFastBlock / 9) * 9 && t < cnt;
    int item = 0;
    double val = 0.0, ri = 0.0, w = 0.0, det = 0.0;
    if (on) {
      item = bin[cap - 1 - t];
      const int l = item % kFastBlock;
      const uint32_t qp = qpair[item];
      const int lf = l / tpf;
      const int u = lf * kc + (int)((qp >> 16) & 63u);
      const int cell = ccell[u];
      const v3 c = mk3(fc[lf][0], fc[lf][1], fc[lf][2]);
      const Tet T{mk3(0, 0, 0), mk3(tv[0][l], tv[1][l], tv[2][l]),
                  mk3(tv[3][l], tv[4][l], tv[5][l]), mk3(tv[6][l], tv[7][l], tv[8][l])};
      det = tv[9][l];
      const int cl = ccls[u] & 7;
      // the four cutting planes in mask order, then the PLIC plane
      const Pl pl = plic_plane_at(s, cell, c);
      const int q0 = ccq0 ? ccq0[u] : m.cf_off[cell];
      uint32_t mm = qp & 0xffffu;
      const Pl a = cell_plane_at(m, q0 + __builtin_ctz(mm), c);
      mm &= mm - 1;
      const Pl b = cell_plane_at(m, q0 + __builtin_ctz(mm), c);
      mm &= mm - 1;
      const Pl d = cell_plane_at(m, q0 + __builtin_ctz(mm), c);
      mm &= mm - 1;
      const Pl e = cell_plane_at(m, q0 + __builtin_ctz(mm), c);
      val = split_term2<5>(dist_table<5>(T, a, b, d, e, pl), i, j, ri);
      w = class_weight(s, cell, cl);
    }
    const double f = (val + __shfl_down(val, 1)) + __shfl_down(val, 2);
    const double ti = ri * f;
    const double tot = (ti + __shfl_down(ti, 3)) + __shfl_down(ti, 6);
    if (on && sub == 0) res[item] = w * (det * tot);
  }
}

// Step 5 on the register path.  A wavefront takes a group of whole geometric
// faces (64 / tets-per-face of them; groups claimed from a counter), one flux
// tet per lane.  First the faces' candidate cells: each face's stencil is
// scanned by all lanes at once and the non-empty cells whose box overlaps
// the flux polyhedron's box are compacted (in stencil order) into LDS with
// their class and box.  Phase A: every tet classifies its face's candidates
// by a mask of the cell planes that cut it; pairs bounded by at most one
// plane are summed at once (a single kept fraction); pairs with two to
// MAXPL planes are queued in LDS bins by plane count, and a tet with a
// pair of more planes (or, without CHUNKED, of a face with more than CAND / F
// candidates; with it the candidates come in chunks of that many, the next
// once the group's tets are through the current one) goes to the general
// kernel's queue; a tet with more than SLOTS queued pairs stops
// at the first that finds its queue full and resumes there in another round
// of the three phases.  Phase B
// evaluates each bin with the plane count uniform across the wave: pairs of
// two planes one lane each (the whole recursion), of three planes one lane
// each on tetrahedral meshes and three lanes each on hexahedral ones, of four
// three lanes each (one per piece of the first plane's split), of five nine
// lanes each (one per piece of the first two splits); phase C adds each tet's
// queued results in stencil order.
// Group g of one list of geometric faces of one mesh (`count` faces at gfaces
// slots first, first + dir, ...; tpf tets per face, F = 64 / tpf per group),
// swept by `sweep` (-s dt).  Must be reached by the whole wave.
template <int SLOTS, int CAND, bool BOXES, int MAXPL, bool CHUNKED>
__device__ __forceinline__ void clip_fast_group(const DMesh &m, const DState &s, const DParams &p,
                                                int g, int count, int first, int dir,
                                                int tpf, double sweep,
                                                unsigned long long &npairs,
                                                unsigned long long &nresc) {
  static_assert(MAXPL <= 4 || !BOXES, "five-plane pairs only for cells that are not boxes");
  // the group's faces: points minus the face centre and their sweeps at the
  // corrected lam, the mean sweep, the point count and the face centre (the
  // apex of the face's tets); every tet is built from these
  __shared__ double fpt[kFacePool][6];  // face fi's point j at fi * (tpf / 5) + j
  __shared__ double fcq[kGroupFaces][3];
  __shared__ int fn[kGroupFaces];
  __shared__ double fc[kGroupFaces][3];
  __shared__ double tv[10][kFastBlock];
  // queued pair: plane mask (bits 0-15), candidate (16-21), box cell (22),
  // plane count - 2 (30-31)
  constexpr int kCap = kFastBlock * SLOTS;
  __shared__ uint32_t qpair[kCap];
  __shared__ double res[kCap];
  // queued pairs by plane count: two planes from the start of bins[0], five
  // from its end, three from the start of bins[1] and four from its end (kCap
  // pairs at most)
  __shared__ uint16_t bins[2][kCap];
  __shared__ int nbin[4];
  // candidates of face fi at fi * (CAND / F) + position
  __shared__ int32_t ccell[CAND];
  __shared__ int8_t ccls[CAND];  // class | 8 for a box cell
  // first plane index (cf_off) of a candidate cell that is not a box
  __shared__ int32_t ccq0[BOXES ? 1 : CAND];
  // candidate bounds (lo x y z, hi x y z): the box test, and the planes of a
  // box cell
  __shared__ double cbox[BOXES ? CAND : 1][6];
  __shared__ double fbox[kGroupFaces][6];
  __shared__ int cnum[kGroupFaces];
  const int lane = threadIdx.x;
  const int F = kFastBlock / tpf;  // faces per group, 1..kGroupFaces
  const int gmax = tpf / 5;        // points per face of the list
  // candidates kept per face (the candidate field of a queued pair has 6 bits)
  const int kc = CAND / F < 63 ? CAND / F : 63;
  {
    if (lane < 4) nbin[lane] = 0;
    // flux polyhedron boxes (points and their swept images) and the faces
    // staged in LDS, one lane per face point: lane fi * padw + j takes point j
    // of face fi, and the face's sums and bounds are butterfly reductions
    // over its padw lanes (every lane of the face ends with the same bits, as
    // the two operands of each addition are the same in every lane).
    // Unpadded: a cell that only touches the box meets the polyhedron in a
    // sliver of zero width (or of the width of the rounding of the tets'
    // vertices), whose volume is below the rounding of the sum.
    {
      const int pw = m.padw;  // 4 or 8
      const int sf = lane / pw, sj = lane - sf * pw;
      const int sslot = g * F + sf;
      const bool sface = sf < F && sslot < count;
      int q = -1;
      double sw = 0.0;
      if (sface) {
        const int f = s.gfaces[(int64_t)first + dir * sslot];
        sw = sweep * s.lam[f];
        q = m.fpad[(int64_t)f * pw + sj];
      }
      v3 x = mk3(0, 0, 0), u = mk3(0, 0, 0);
      v3 lo = mk3(1e300, 1e300, 1e300), hi = mk3(-1e300, -1e300, -1e300);
      if (q >= 0) {
        const PointRec pr = point_rec(s.XU, q);
        x = pr.x;
        u = sw * pr.u;
        const v3 y = x + u;
        lo = mk3(dmin(x.x, y.x), dmin(x.y, y.y), dmin(x.z, y.z));
        hi = mk3(dmax(x.x, y.x), dmax(x.y, y.y), dmax(x.z, y.z));
      }
      const unsigned long long has = __ballot(q >= 0);
      const int n = (int)__popcll((has >> (sf * pw)) & ((1ull << pw) - 1ull));
      v3 c = x, cs = u;
      for (int o = 1; o < pw; o <<= 1) {
        c = c + mk3(__shfl_xor(c.x, o), __shfl_xor(c.y, o), __shfl_xor(c.z, o));
        cs = cs + mk3(__shfl_xor(cs.x, o), __shfl_xor(cs.y, o), __shfl_xor(cs.z, o));
        lo = mk3(dmin(lo.x, __shfl_xor(lo.x, o)), dmin(lo.y, __shfl_xor(lo.y, o)),
                 dmin(lo.z, __shfl_xor(lo.z, o)));
        hi = mk3(dmax(hi.x, __shfl_xor(hi.x, o)), dmax(hi.y, __shfl_xor(hi.y, o)),
                 dmax(hi.z, __shfl_xor(hi.z, o)));
      }
      if (q >= 0) {
        c = (1.0 / n) * c;
        cs = (1.0 / n) * cs;  // mean sweep
        if (n <= gmax) {  // always, by the list the face is on
          double *row = fpt[sf * gmax + sj];
          row[0] = x.x - c.x; row[1] = x.y - c.y; row[2] = x.z - c.z;
          row[3] = u.x; row[4] = u.y; row[5] = u.z;
        }
        if (sj == 0) {
          fn[sf] = n;
          fc[sf][0] = c.x; fc[sf][1] = c.y; fc[sf][2] = c.z;
          fcq[sf][0] = cs.x; fcq[sf][1] = cs.y; fcq[sf][2] = cs.z;
          fbox[sf][0] = lo.x; fbox[sf][1] = lo.y; fbox[sf][2] = lo.z;
          fbox[sf][3] = hi.x; fbox[sf][4] = hi.y; fbox[sf][5] = hi.z;
        }
      }
    }
    __syncthreads();
    // phase A
    const int fi = lane / tpf, k = lane - fi * tpf;
    const int slot = g * F + fi;
    const bool active = fi < F && slot < count;
    const int64_t idx = ((int64_t)first + dir * slot) * m.tpf + k;
    bool defer = false, live = false;
    double acc = 0.0, sgn = 1.0;
    if (active) {
      v3 t1, t2, t3;
      double det;
      live = !p.check_stencil &&
             staged_tet(&fpt[fi * gmax], fn[fi], fcq[fi], k, t1, t2, t3, det, sgn);
      defer = p.check_stencil;
      if (live && !defer) {
        tv[0][lane] = t1.x; tv[1][lane] = t1.y; tv[2][lane] = t1.z;
        tv[3][lane] = t2.x; tv[4][lane] = t2.y; tv[5][lane] = t2.z;
        tv[6][lane] = t3.x; tv[7][lane] = t3.y; tv[8][lane] = t3.z;
        tv[9][lane] = det;
      }
    }
    if (defer) live = false;
    bool todo = live;   // candidates of the current chunk left to visit
    bool more = false;  // candidates past the current chunk left to visit
    int ci0 = 0;
    unsigned long long np = 0;
    // candidate cells of the group's faces in chunks of kc per face (in
    // stencil order, kFastBlock / F lanes per face): a face with more takes
    // the next chunk once its tets are through the current one
    for (int skip = 0;; skip += kc) {
      {
        const int L = kFastBlock / F;
        const int cf = lane / L, e_in = lane - cf * L;
        const int slot = g * F + cf;
        const bool mine = cf < F && slot < count;
        int w = 0, nst = 0;
        if (mine) {
          const int f = s.gfaces[(int64_t)first + dir * slot];
          w = m.st_off[f];
          nst = m.st_off[f + 1] - w;
        }
        int most = nst;  // the largest stencil of the group sets the trip count
        for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
        const unsigned long long seg =
            !mine ? 0ull : (L == kFastBlock ? ~0ull : (((1ull << L) - 1ull) << (cf * L)));
        int cnt = 0;
        for (int e0 = 0; e0 < most; e0 += L) {
          const int e = e0 + e_in;
          bool keep = false;
          int cell = 0, cl = 0;
          double4 blo = make_double4(0, 0, 0, 0), bhi = blo;
          if (mine && e < nst) {
            cell = m.st[w + e];
            cl = s.cls[cell];
            if (cl != 0) {
              blo = m.bblo[cell];
              bhi = m.bbhi[cell];
              keep = !(fbox[cf][3] <= blo.x || fbox[cf][0] >= bhi.x || fbox[cf][4] <= blo.y ||
                       fbox[cf][1] >= bhi.y || fbox[cf][5] <= blo.z || fbox[cf][2] >= bhi.z);
            }
          }
          const unsigned long long bal = __ballot(keep) & seg;
          const int pos = cnt + (int)__popcll(bal & ((1ull << lane) - 1ull));
          if (keep && pos >= skip && pos < skip + kc) {
            const int u = cf * kc + (pos - skip);
            ccell[u] = cell;
            ccls[u] = (int8_t)(cl | (BOXES && m.isbox[cell] ? 8 : 0));
            if (!BOXES) ccq0[u] = m.cf_off[cell];
            if (BOXES) {
              cbox[u][0] = blo.x;
              cbox[u][1] = blo.y;
              cbox[u][2] = blo.z;
              cbox[u][3] = bhi.x;
              cbox[u][4] = bhi.y;
              cbox[u][5] = bhi.z;
            }
          }
          cnt += (int)__popcll(bal);
        }
        if (mine && e_in == 0) cnum[cf] = cnt;
      }
      __syncthreads();
      // without chunks, a face with more candidates than its share goes to
      // the general kernel
      if constexpr (!CHUNKED) {
        if (todo && cnum[fi] > kc) {
          defer = true;
          live = todo = false;
        }
      }
      // Phase A1, for cells that are not boxes: which candidates of its face
      // may overlap each tet (bit ci of cmask), found with the lanes over the
      // candidates (each loads its cell's bounds and planes once) and a loop
      // over the face's tets (their vertices read from LDS).  The tests are
      // those of pair_cuts_box in the same arithmetic, so phase A visits the
      // pairs it would keep and skips the rest without loading anything; the
      // first round of phase A also takes each pair's cutting-plane mask from
      // A1 (a code byte per tet and candidate: 0x80 overlap, bits 0-3 the
      // mask of the first four planes, 0x10 a cell of more planes, whose pair
      // is tested again).  The tables live in res, which phase B fills only
      // later.
      unsigned long long cmask = ~0ull;
      uint8_t *tcode = reinterpret_cast<uint8_t *>(res + kFastBlock);
      static_assert(BOXES || 8 * kFastBlock + kFastBlock * 63 <= 8 * kCap, "A1 tables in res");
      if constexpr (!BOXES) {
        unsigned long long *tmask = reinterpret_cast<unsigned long long *>(res);
        tmask[lane] = 0ull;
        const int L = kFastBlock / F;  // lanes per face
        const int cf = lane / L, cin = lane - cf * L;
        const bool fok = cf < F && g * F + cf < count;
        const int ncf = fok ? min(cnum[cf] - skip, kc) : 0;
        int mostc = ncf;
        for (int o = 32; o > 0; o >>= 1) mostc = max(mostc, __shfl_xor(mostc, o));
        const unsigned long long seg = L >= 64 ? ~0ull : ((1ull << L) - 1ull);
        const v3 cc = fok ? mk3(fc[cf][0], fc[cf][1], fc[cf][2]) : mk3(0, 0, 0);
        __syncthreads();
        for (int c0 = 0; c0 < mostc; c0 += L) {
          const int ci = c0 + cin;
          const bool has = ci < ncf;
          int np = 0, q0 = 0;
          double4 blo = make_double4(0, 0, 0, 0), bhi = blo;
          Pl cp[4] = {Pl{0, 0, 0, 0}, Pl{0, 0, 0, 0}, Pl{0, 0, 0, 0}, Pl{0, 0, 0, 0}};
          if (has) {
            const int u = cf * kc + ci;
            const int cell = ccell[u];
            q0 = ccq0[u];
            blo = m.bblo[cell];
            bhi = m.bbhi[cell];
            np = m.npl[cell];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (j < np) cp[j] = cell_plane_at(m, q0 + j, cc);
          }
          for (int k = 0; k < tpf; ++k) {
            bool hit = false;
            uint32_t cut = 0;
            const int t = cf * tpf + k;
            if (has) {
              const v3 t1 = mk3(tv[0][t], tv[1][t], tv[2][t]);
              const v3 t2 = mk3(tv[3][t], tv[4][t], tv[5][t]);
              const v3 t3 = mk3(tv[6][t], tv[7][t], tv[8][t]);
              v3 lo, hi;
              tet_bbox(cc, t1, t2, t3, lo, hi);
              hit = !(hi.x <= blo.x || lo.x >= bhi.x || hi.y <= blo.y || lo.y >= bhi.y ||
                      hi.z <= blo.z || lo.z >= bhi.z);
              // plane j: false when the tet lies outside it, else its cut bit
              auto test = [&](const Pl &pl, int j) {
                const v3 nn = mk3(pl.x, pl.y, pl.z);
                const double off = pl.w;
                const double d1 = off - dot(nn, t1), d2 = off - dot(nn, t2),
                             d3 = off - dot(nn, t3);
                const double dmx = dmax(dmax(off, d1), dmax(d2, d3));
                const double dmn = dmin(dmin(off, d1), dmin(d2, d3));
                cut |= (dmn < 0.0 ? 1u : 0u) << (j & 3);
                return dmx > 0.0;
              };
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (hit && j < np && !test(cp[j], j)) hit = false;
              for (int j = 4; hit && j < np; ++j)
                if (!test(cell_plane_at(m, q0 + j, cc), j)) hit = false;
              tcode[t * kc + ci] = (uint8_t)(hit ? 0x80u | (cut & 15u) | (np > 4 ? 0x10u : 0u) : 0u);
            }
            const unsigned long long b = __ballot(hit);
            if (fok && cin == 0) tmask[cf * tpf + k] |= ((b >> (cf * L)) & seg) << c0;
          }
        }
        __syncthreads();
        cmask = tmask[lane];
      }
      // Phases A to C in rounds: a tet whose queue is full stops at that pair
      // and resumes there in the next round, once its queued pairs are added.
      bool first = true;  // A1's code bytes are valid (res not yet written)
      for (;;) {
        int nq = 0;
        if (todo) {
          // the tet from its LDS row (kept there for phase B anyway)
          const v3 c = mk3(fc[fi][0], fc[fi][1], fc[fi][2]);
          const v3 t1 = mk3(tv[0][lane], tv[1][lane], tv[2][lane]);
          const v3 t2 = mk3(tv[3][lane], tv[4][lane], tv[5][lane]);
          const v3 t3 = mk3(tv[6][lane], tv[7][lane], tv[8][lane]);
          const double det = tv[9][lane];
          const Tet T{mk3(0, 0, 0), t1, t2, t3};
          v3 lo, hi;
          tet_bbox(c, t1, t2, t3, lo, hi);
          const int nc = min(cnum[fi] - skip, kc);
          bool paused = false, inside = false;
          int ci = ci0;
          for (; ci < nc; ++ci) {
            if constexpr (!BOXES) {  // on to the next candidate phase A1 kept
              const unsigned long long r = cmask >> ci;
              if (!r) break;
              ci += __builtin_ctzll(r);
            }
            const int u = fi * kc + ci;
            const int cell = ccell[u];
            const int cb = ccls[u];
            const int cl = cb & 7;
            const bool box = BOXES && (cb & 8);
            const double *bb = cbox[BOXES ? u : 0];
            uint32_t mask;
            int ncut;
            uint32_t code = 0;
            if (!BOXES && first) code = tcode[lane * kc + ci];
            if (!BOXES && (code & 0x90u) == 0x80u) {
              mask = code & 15u;
              ncut = __builtin_popcount(mask);
            } else if (!BOXES) ncut = pair_cuts(m, c, T, lo, hi, cell, mask);
            else if (box) ncut = box_cuts(bb, c, T, mask);
            else
              ncut = pair_cuts_box(m, c, T, lo, hi, mk3(bb[0], bb[1], bb[2]),
                                   mk3(bb[3], bb[4], bb[5]), cell, mask);
            if (ncut < 0) continue;
            ++np;
            // next to cell planes, the PLIC plane of an interface cell counts
            // only where it crosses the tet: with the tet wholly on its kept
            // side it drops out, wholly beyond it the pair holds no phase
            bool plic = cl == 1;
            if (plic && ncut > 0) {
              const D4 dp = plane_dists(T, plic_plane_at(s, cell, c));
              if (dmax(dmax(dp.a, dp.b), dmax(dp.c, dp.d)) <= 0.0) continue;
              if (dmin(dmin(dp.a, dp.b), dmin(dp.c, dp.d)) >= 0.0) plic = false;
            }
            const int npl = ncut + (plic ? 1 : 0);
            if (npl <= 1) {
              double fr = 1.0;
              if (npl == 1) {
                const int q = __builtin_ctz(mask);
                const Pl pl = !ncut ? plic_plane_at(s, cell, c)
                                    : (box ? box_plane(bb, q, c)
                                           : cell_plane_at(m, (BOXES ? m.cf_off[cell] : ccq0[u]) + q,
                                                           c));
                fr = tet_kept_fraction(plane_dists(T, pl));
              }
              acc += class_weight(s, cell, cl) * det * fr;
            } else if (npl > MAXPL) {
              defer = true;
              break;
            } else if (nq == SLOTS) {
              --np;  // counted again when the next round takes it
              paused = true;
              break;
            } else {
              qpair[nq * kFastBlock + lane] = mask | ((uint32_t)ci << 16) | (box ? 1u << 22 : 0u) |
                                              ((uint32_t)(npl - 2) << 30);
              ++nq;
            }
            if (ncut == 0) {  // the tet lies inside this cell
              inside = true;
              break;
            }
          }
          if (defer) live = false;
          todo = live && paused;
          more = CHUNKED && live && !paused && !inside && cnum[fi] > skip + kc;
          ci0 = todo ? ci : 0;
          if (live) {
            for (int j = 0; j < nq; ++j) {
              int b = (int)(qpair[j * kFastBlock + lane] >> 30);
              int pos = atomicAdd(&nbin[b], 1);
              if (b >= 2) pos = kCap - 1 - pos;
              bins[b == 0 || b == 3 ? 0 : 1][pos] = (uint16_t)(j * kFastBlock + lane);
            }
          }
        }
        __syncthreads();
        // phase B, one bin at a time (the plane count uniform across the wave):
        // pairs of two planes one lane each, of three planes three lanes each
        // (one each on tetrahedral meshes, whose bins are fuller), of four three
        // lanes each.  Every bin takes the same way whatever its size: which
        // faces share a group follows the order of the geometric-face list,
        // which is not fixed from run to run.
        const int32_t *q0s = BOXES ? nullptr : ccq0;
        one_lane_bin<2>(m, s, qpair, tv, fc, ccell, ccls, q0s, cbox, tpf, kc, bins[0], nbin[0],
                        false, kCap, res);
        if constexpr (BOXES)
          three_lane_bin<3>(m, s, qpair, tv, fc, ccell, ccls, q0s, cbox, tpf, kc, bins[1],
                            nbin[1], false, kCap, res);
        else
          one_lane_bin<3>(m, s, qpair, tv, fc, ccell, ccls, q0s, cbox, tpf, kc, bins[1], nbin[1],
                          false, kCap, res);
        three_lane_bin<4>(m, s, qpair, tv, fc, ccell, ccls, q0s, cbox, tpf, kc, bins[1], nbin[2],
                          true, kCap, res);
        if constexpr (MAXPL >= 5)
          nine_lane_bin(m, s, qpair, tv, fc, ccell, ccls, q0s, tpf, kc, bins[0], nbin[3], kCap,
                        res);
        __syncthreads();
        // phase C
        first = false;
        if (live)
          for (int j = 0; j < nq; ++j) acc += res[j * kFastBlock + lane];
        if (!__ballot(todo)) break;
        if (lane < 4) nbin[lane] = 0;
        __syncthreads();
      }
      if (!__ballot(more)) break;
      if (lane == 0) ++nresc;  // the group's stencils scanned again for the next chunk
      todo = more;
      more = false;
      ci0 = 0;
      if (lane < 4) nbin[lane] = 0;
      __syncthreads();
    }
    if (live) {
      npairs += np;
      s.tetvol[idx] = sgn * acc / 6.0;
    } else if (active && !defer) {
      s.tetvol[idx] = 0.0;
    }
    int q = wave_append(&s.work[kWDeferred], defer);
    if (defer) s.defer[q] = (int32_t)idx;
    __syncthreads();
  }
}

// Step 5 on the register path over one mesh: groups are taken kClaim at a
// time, the first kClaim by block index, the rest claimed from a counter
// (thousands of waves claiming one group each serialise on the counter's
// atomic, above all at the start of the kernel).
template <int SLOTS, int CAND, bool BOXES, int MAXPL, bool CHUNKED>
__global__ __launch_bounds__(kFastBlock) __attribute__((amdgpu_waves_per_eu(BOXES ? 3 : 2)))
void k_clip_fast(DMesh m, DState s, DParams p) {
  __shared__ int group;
  const int lane = threadIdx.x;
  const int step = *s.stepno;
  const double sweep = -s.sc[step] * s.dt[step];
  const ClipGroups cg = clip_groups(m, s);
  const int ngroups = cg.total;
  unsigned long long npairs = 0, nresc = 0;
  int left = -1;
  for (;;) {
    if (lane == 0) {
      if (left < 0) {
        group = kClaim * (int)blockIdx.x;
        left = kClaim;
      } else if (left == 0) {
        group = kClaim * ((int)gridDim.x + atomicAdd(&s.work[kWClipNext], 1));
        left = kClaim;
      } else {
        group = group + 1;
      }
      --left;
    }
    __syncthreads();
    const int g = group;
    if (g >= ngroups) break;
    // one call site for both lists (the group body is inlined once)
    const bool sm = g < cg.nsmall;
    clip_fast_group<SLOTS, CAND, BOXES, MAXPL, CHUNKED>(
        m, s, p, sm ? g : g - cg.nsmall, sm ? cg.na : cg.nb, sm ? 0 : (int)m.nf - 1,
        sm ? 1 : -1, sm ? cg.tsmall : m.tpf, sweep, npairs, nresc);
  }
  wave_count(cnt_at(s.cnt, kCntPairs), npairs);
  wave_count(cnt_at(s.cnt, kCntRescans), nresc);
}

// General clip of the queued tets, kGenTets tets per wave with kGenLanes lanes
// each over the face's stencil cells: closed forms up to kRegPlanes planes per
// pair in every lane at once; the rare pairs with more planes then take turns
// on one vertex-graph polytope in LDS shared by the wave.  A tet's pair
// volumes are added lane by lane in stencil order (the same order on every
// run).
// The deferred tets i0 .. i0 + kGenTets - 1 (of `count`) of one mesh.
__device__ __forceinline__ void clip_general_tets(const DMesh &m, const DState &s,
                                                  const DParams &p, int i0, int count, double dt,
                                                  double sc, unsigned long long &ncap,
                                                  unsigned long long &npairs) {
  __shared__ double lx[kPolyCap], ly[kPolyCap], lz[kPolyCap], ld[kPolyCap];
  __shared__ uint8_t lnb[3 * kPolyCap], laux[kPolyCap];
  static_assert(kClipBlock == 64, "one wave per block");
  const int lane = threadIdx.x;
  Poly P;
  P.px = lx; P.py = ly; P.pz = lz; P.ps = ld;
  P.nb = lnb; P.aux = laux;
  P.st = 1; P.cap = kPolyCap; P.nv = 0;

  __shared__ double red[2][kClipBlock];
  // pairs of four planes handed back by the lanes: distances, weight, det,
  // and the kept fraction, evaluated by three lanes each (one per piece of
  // the first plane's split)
  __shared__ double fd[kClipBlock][20];
  __shared__ double fw[kClipBlock], fres[kClipBlock];
  __shared__ int8_t fidx[kClipBlock], fidx5[kClipBlock];
  // kGenTets tets per wavefront, kGenLanes lanes each over the tet's stencil
  const int seg = lane / kGenLanes, sl = lane - seg * kGenLanes;
  {
    const int i = i0 + seg;
    const bool mine = seg < kGenTets && i < count;
    int64_t idx = 0;
    int f = 0;
    v3 c = mk3(0, 0, 0), t1 = c, t2 = c, t3 = c;
    double det = 0.0, sgn = 1.0;
    bool live = false;
    int e0 = 0, e1 = 0;
    if (mine) {
      idx = s.defer[i];
      const int slot = (int)(idx / m.tpf);
      const int k = (int)(idx - (int64_t)slot * m.tpf);
      f = s.gfaces[slot];
      live = flux_tet(m, s, dt, sc, f, k, c, t1, t2, t3, det, sgn);
      if (live) {
        e0 = m.st_off[f];
        e1 = m.st_off[f + 1];
      }
    }
    // the largest stencil among the wave's tets sets the trip count
    int most = e1 - e0;
    for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
    const Tet T{mk3(0, 0, 0), t1, t2, t3};
    v3 lo, hi;
    tet_bbox(c, t1, t2, t3, lo, hi);
    double a = 0.0, cv = 0.0;
    for (int b = 0; b < most; b += kGenLanes) {
      const int e = e0 + b + sl;
      const bool act = live && e < e1;
      double v = 0.0, vc = 0.0;
      Four four;
      four.row = fd[lane];
      four.on = false;
      if (act)
        v = pair_phase6(m, s, p, c, T, det, lo, hi, m.st[e], P, ncap, npairs, &vc, false, &four);
      // pairs of four planes listed in LDS, three lanes per pair; pairs of
      // five, nine lanes per pair (one per piece of the first two splits)
      const unsigned long long fm = __ballot(four.on);
      if (fm) {
        const unsigned long long m4 = __ballot(four.on && !four.five);
        const unsigned long long m5 = fm & ~m4;
        const unsigned long long below = (1ull << lane) - 1ull;
        if (four.on) {
          if (four.five) fidx5[__popcll(m5 & below)] = (int8_t)lane;
          else fidx[__popcll(m4 & below)] = (int8_t)lane;
          fw[lane] = four.w;
        }
        __syncthreads();
        const int nf4 = (int)__popcll(m4);
        for (int b4 = 0; b4 < nf4; b4 += kClipBlock / 3) {
          const int pr = b4 + lane / 3, piece = lane % 3;
          double val = 0.0;
          if (lane < (kClipBlock / 3) * 3 && pr < nf4) {
            const double *q = fd[fidx[pr]];
            const TD<4> D{{{q[0], q[1], q[2], q[3]}}, {{q[4], q[5], q[6], q[7]}},
                          {{q[8], q[9], q[10], q[11]}}, {{q[12], q[13], q[14], q[15]}}};
            const Split<4> sp = split_first<4>(D);
            if (piece < sp.n) {
              double r;
              const TD<3> Pc = split_piece<4>(sp, piece, r);
              val = r * kept_fraction<3>(Pc);
            }
          }
          const double v1 = __shfl_down(val, 1), v2 = __shfl_down(val, 2);
          if (piece == 0 && lane < (kClipBlock / 3) * 3 && pr < nf4)
            fres[fidx[pr]] = (val + v1) + v2;
        }
        const int nf5 = (int)__popcll(m5);
        for (int b5 = 0; b5 < nf5; b5 += kClipBlock / 9) {
          const int pr = b5 + lane / 9, sub = lane % 9;
          const bool on5 = lane < (kClipBlock / 9) * 9 && pr < nf5;
          double val = 0.0, ri = 0.0;
          if (on5) {
            const double *q = fd[fidx5[pr]];
            const TD<5> D{{{q[0], q[1], q[2], q[3], q[4]}}, {{q[5], q[6], q[7], q[8], q[9]}},
                          {{q[10], q[11], q[12], q[13], q[14]}},
                          {{q[15], q[16], q[17], q[18], q[19]}}};
            val = split_term2<5>(D, sub / 3, sub % 3, ri);
          }
          const double f = (val + __shfl_down(val, 1)) + __shfl_down(val, 2);
          const double ti = ri * f;
          const double tot = (ti + __shfl_down(ti, 3)) + __shfl_down(ti, 6);
          if (on5 && sub == 0) fres[fidx5[pr]] = tot;
        }
        __syncthreads();
        if (four.on) v = fw[lane] * (det * fres[lane]);
        __syncthreads();
      }
      const bool pend = act && v != v;
      unsigned long long pm = __ballot(pend);
      while (pm) {
        const int L = __ffsll((long long)pm) - 1;
        pm &= pm - 1ull;
        // the polytope changes hands: order one lane's LDS traffic before
        // the next lane's (without this the compiler may interleave them)
        __syncthreads();
        if (lane == L)
          v = pair_phase6(m, s, p, c, T, det, lo, hi, m.st[e], P, ncap, npairs, &vc, true);
      }
      __syncthreads();
      a += v;
      cv += vc;
    }
    // per tet, its lanes' sums added in lane order
    red[0][lane] = a;
    red[1][lane] = cv;
    __syncthreads();
    if (mine && sl == 0) {
      double acc = 0.0, cover = 0.0;
      for (int j = 0; j < kGenLanes; ++j) {
        acc += red[0][lane + j];
        cover += red[1][lane + j];
      }
      s.tetvol[idx] = live ? sgn * acc / 6.0 : 0.0;
      if (p.check_stencil) {
        s.tetdef[idx] = live ? sgn * (det - cover) / 6.0 : 0.0;
        s.tetgross[idx] = live ? det / 6.0 : 0.0;
      }
    }
    __syncthreads();
  }
}

// the counters of the general clip, and the capacity flag
__device__ __forceinline__ void clip_general_counts(const DState &s, unsigned long long ncap,
                                                    unsigned long long npairs) {
  wave_count(cnt_at(s.cnt, kCntCapacity), ncap);
  wave_count(cnt_at(s.cnt, kCntPairs), npairs);
  if (__ballot(ncap != 0) && lane_id() == 0) flag(s.flags, kFlagCapacity);
}

__global__ __launch_bounds__(kClipBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_clip_general(DMesh m, DState s, DParams p) {
  const int step = *s.stepno;
  const double dt = s.dt[step], sc = s.sc[step];
  const int count = s.work[kWDeferred];
  unsigned long long ncap = 0, npairs = 0;
  for (int i0 = blockIdx.x * kGenTets; i0 < count; i0 += gridDim.x * kGenTets)
    clip_general_tets(m, s, p, i0, count, dt, sc, ncap, npairs);
  clip_general_counts(s, ncap, npairs);
}

// Sum of the tets of each geometric face.  With check_stencil: the uncovered
// signed volume of the face must vanish to 1e-12 of max(gross tet volume,
// owner cell volume).
__device__ __forceinline__ void face_sum_one(const DMesh &m, const DState &s, const DParams &p,
                                             int i, int na, unsigned long long &nleak) {
  {
    const int64_t sl = geo_slot(m, na, i);
    const double *tv = s.tetvol + sl * m.tpf;
    const int f = s.gfaces[sl];
    const int nt = 5 * (m.foff[f + 1] - m.foff[f]);  // the face's tets
    double acc = 0.0;
    // five tets per point of the face: the loads of a point's five go together
    for (int k = 0; k < nt; k += 5) {
      const double w0 = tv[k], w1 = tv[k + 1], w2 = tv[k + 2], w3 = tv[k + 3], w4 = tv[k + 4];
      acc += w0;
      acc += w1;
      acc += w2;
      acc += w3;
      acc += w4;
    }
    if (s.fstatus[f]) acc *= s.vscale[f];
    s.vphase[f] = acc;
    if (p.check_stencil) {
      double dsum = 0.0, gsum = 0.0;
      for (int k = 0; k < nt; ++k) {
        dsum += s.tetdef[sl * m.tpf + k];
        gsum += s.tetgross[sl * m.tpf + k];
      }
      if (fabs(dsum) > 1e-12 * dmax(gsum, m.V[m.own[f]])) ++nleak;
    }
  }
}
__device__ __forceinline__ void face_sum_counts(const DState &s, unsigned long long nleak) {
  wave_count(cnt_at(s.cnt, kCntLeaks), nleak);
  if (__ballot(nleak != 0) && lane_id() == 0) flag(s.flags, kFlagLeak);
}
__global__ __launch_bounds__(kBlock) void k_face_sum(DMesh m, DState s, DParams p) {
  const int count = geo_count(s), na = s.work[kWGeometric];
  unsigned long long nleak = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    face_sum_one(m, s, p, i, na, nleak);
  face_sum_counts(s, nleak);
}

// alpha_c^{n+1} = alpha_c^n - (1/V_c) sum_f sgn_cf V_{f,alpha}, every cell
// (and each block's sum of the phase volumes through its cells' boundary
// faces, the first stage of the ledger);
// with the narrow band (Section 2.3) every cell but the bulk cells, those
// whose faces' points touch only cells that are exactly 0 (or only exactly 1),
// so that every cell sharing a point with them is.  With wisps on, the
// updated cells outside the interface band whose alpha is not exactly 0 or
// 1 are listed with their excess over the nearer of the two.
// Block vb of the update of one mesh: cells vb * kBlock ... (and the block's
// part of the ledger in part[vb]).
__device__ __forceinline__ void update_blk(const DMesh &m, const DState &s, const DParams &p,
                                           int64_t vb) {
  __shared__ double red[kBlock];
  int64_t c = vb * (int64_t)blockDim.x + threadIdx.x;
  const uint32_t stamp = p.wisps ? s.wctr[0] + 1u : 0u;
  bool wisp = false;
  double ex = 0.0;
  double led = 0.0;  // phase volume through the cell's boundary faces
  if (c < m.nc) {
    const int k0 = m.cf_off[c], k1 = m.cf_off[c + 1];
    bool skip = false;
    if (p.band) {
      uint8_t b = 3;
#pragma unroll 6
      for (int k = k0; k < k1; ++k) {
        int sf = m.cf[k];
        b &= s.fbulk[sf >= 0 ? sf : ~sf];
      }
      skip = b != 0;
      if (skip) {
        for (int k = k0; k < k1; ++k) {
          const int sf = m.cf[k];
          if (sf >= m.ni) led += s.vphase[sf];
        }
      }
    }
    if (!skip) {
      double acc = 0.0;
      // unrolled so that the face ids, then the phase volumes, load together
#pragma unroll 6
      for (int k = k0; k < k1; ++k) {
        const int sf = m.cf[k];
        const double v = s.vphase[sf >= 0 ? sf : ~sf];
        acc += sf >= 0 ? v : -v;
        led += sf >= m.ni ? v : 0.0;
      }
      const double V = m.V[c];
      const double a = s.alpha[c] - acc / V;
      s.alpha[c] = a;
      if (p.wisps && !(a > p.eps && a < 1.0 - p.eps) && a != 0.0 && a != 1.0) {
        wisp = true;
        ex = (a - (a <= p.eps ? 0.0 : 1.0)) * V;
      }
    }
  }
  if (p.wisps) {
    int slot = block_append(&s.work[kWWisps], wisp);
    if (wisp) {
      s.wlist[slot] = (int32_t)c;
      s.wex[c] = ex;
      s.wstamp[c] = stamp;
    }
  }
  // the block's part of the boundary ledger, summed in a fixed order
  red[threadIdx.x] = led;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) s.part[vb] = red[0];
  __syncthreads();  // red is reused by the next block of a persistent caller
}
__global__ __launch_bounds__(kBlock) void k_update(DMesh m, DState s, DParams p) {
  update_blk(m, s, p, blockIdx.x);
}

// ---------------------------------------------------------------------------
// wisp redistribution (Section 2.3), four passes over this step's wisps and
// their receivers (interface cells sharing a point with a wisp):
//   receivers   each wisp lists the interface cells around it, once each
//   offers      per receiver r: rho+ = (1 - eps - alpha_r) V_r / sum of the
//               positive excesses around it, rho- = (alpha_r - eps) V_r / sum
//               of the negative ones (the offer to wisp w is rho |m_w|)
//   sums        per wisp: the sum of its receivers' rho of its sign; it moves
//               |m_w| min(1, sum), a share rho / sum to each receiver
//   moves       per receiver: alpha += sum_w m_w rho min(1, 1 / sum_w) / V;
//               per wisp: alpha = target if sum >= 1, else alpha - m sum / V
// One wavefront per wisp or receiver, lanes over its point neighbours, sums by
// butterfly (a fixed order).  Receivers and wisps are disjoint (inside and
// outside the interface band), so the last pass reads and writes each cell's
// alpha from one wavefront only.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_band(double a, double eps) { return a > eps && a < 1.0 - eps; }

__device__ __forceinline__ int wave_index() {
  return (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
}
__device__ __forceinline__ int wave_stride() { return (int)(gridDim.x * (blockDim.x / kWave)); }

__global__ __launch_bounds__(kBlock) void k_wisp_receivers(DMesh m, DState s, DParams p) {
  const int count = s.work[kWWisps];
  const uint32_t stamp = s.wctr[0] + 1u;
  const int lane = lane_id();
  for (int i = wave_index(); i < count; i += wave_stride()) {
    const int w = s.wlist[i];
    const int k1 = m.cpn_off[w + 1];
    for (int k = m.cpn_off[w] + lane; k - lane < k1; k += kWave) {
      bool fresh = false;
      int r = 0;
      if (k < k1) {
        r = m.cpn[k];
        // the plain read skips the atomic for receivers stamped already
        fresh = in_band(s.alpha[r], p.eps) && s.rstamp[r] != stamp &&
                atomicExch(&s.rstamp[r], stamp) != stamp;
      }
      const int slot = wave_append(&s.work[kWRecv], fresh);
      if (fresh) s.rlist[slot] = r;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_wisp_offers(DMesh m, DState s, DParams p) {
  const int count = s.work[kWRecv];
  const uint32_t stamp = s.wctr[0] + 1u;
  const int lane = lane_id();
  for (int i = wave_index(); i < count; i += wave_stride()) {
    const int r = s.rlist[i];
    const int k1 = m.cpn_off[r + 1];
    double pos = 0.0, neg = 0.0;
    for (int k = m.cpn_off[r] + lane; k < k1; k += kWave) {
      const int w = m.cpn[k];
      if (s.wstamp[w] != stamp) continue;
      const double e = s.wex[w];
      if (e > 0.0) pos += e;
      else neg -= e;
    }
    pos = wave_sum_d(pos);
    neg = wave_sum_d(neg);
    if (lane == 0) {
      const double a = s.alpha[r], V = m.V[r];
      s.rho[r] = make_double2(pos > 0.0 ? (1.0 - p.eps - a) * V / pos : 0.0,
                              neg > 0.0 ? (a - p.eps) * V / neg : 0.0);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_wisp_sums(DMesh m, DState s, DParams p) {
  const int count = s.work[kWWisps];
  const int lane = lane_id();
  unsigned long long nleft = 0;
  for (int i = wave_index(); i < count; i += wave_stride()) {
    const int w = s.wlist[i];
    const bool give = s.wex[w] > 0.0;
    const int k1 = m.cpn_off[w + 1];
    double sum = 0.0;
    for (int k = m.cpn_off[w] + lane; k < k1; k += kWave) {
      const int r = m.cpn[k];
      if (!in_band(s.alpha[r], p.eps)) continue;
      const double2 rr = s.rho[r];
      sum += give ? rr.x : rr.y;
    }
    sum = wave_sum_d(sum);
    if (lane == 0) {
      s.wsum[w] = sum;
      nleft += sum < 1.0;
    }
  }
  wave_count(cnt_at(s.cnt, kCntWispsLeft), nleft);
}

__global__ __launch_bounds__(kBlock) void k_wisp_moves(DMesh m, DState s, DParams p) {
  const int nr = s.work[kWRecv], nw = s.work[kWWisps];
  const uint32_t stamp = s.wctr[0] + 1u;
  const int lane = lane_id();
  for (int i = wave_index(); i < nr + nw; i += wave_stride()) {
    if (i < nr) {
      const int r = s.rlist[i];
      const double2 rr = s.rho[r];
      const int k1 = m.cpn_off[r + 1];
      double gain = 0.0;
      for (int k = m.cpn_off[r] + lane; k < k1; k += kWave) {
        const int w = m.cpn[k];
        if (s.wstamp[w] != stamp) continue;
        const double e = s.wex[w], sum = s.wsum[w];
        gain += e * (e > 0.0 ? rr.x : rr.y) * (sum > 1.0 ? 1.0 / sum : 1.0);
      }
      gain = wave_sum_d(gain);
      if (lane == 0) s.alpha[r] += gain / m.V[r];
    } else if (lane == 0) {
      const int w = s.wlist[i - nr];
      const double a = s.alpha[w], sum = s.wsum[w];
      s.alpha[w] = sum >= 1.0 ? (a <= p.eps ? 0.0 : 1.0) : a - s.wex[w] * sum / m.V[w];
    }
  }
}

// boundary ledger, second stage: one block adds the update kernel's
// per-block sums in a fixed order, and the step's counts
__device__ __forceinline__ void ledger_blk(const DMesh &m, const DState &s, const DParams &p,
                                           int nparts) {
  __shared__ double red[kLedgerBlock];
  double acc = 0.0;
  // unrolled so that a thread's partial sums load together
#pragma unroll 8
  for (int i = threadIdx.x; i < nparts; i += kLedgerBlock) acc += s.part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kLedgerBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s.ledger[0] += red[0];
    *cnt_at(s.cnt, kCntSteps) += 1;
    *cnt_at(s.cnt, kCntGeometric) += (unsigned long long)geo_count(s);
    *cnt_at(s.cnt, kCntInterface) += (unsigned long long)s.work[kWInterface];
    *cnt_at(s.cnt, kCntDeferred) += (unsigned long long)s.work[kWDeferred];
    if (p.wisps) {
      *cnt_at(s.cnt, kCntWisps) += (unsigned long long)s.work[kWWisps];
      s.wctr[0] += 1u;  // the next step's wisps and receivers get a new stamp
    }
    s.stepno[0] += 1;  // the next step reads dt, scale at the next index
    for (int w = 0; w < kWNum; ++w) s.work[w] = 0;  // the next step's lists start empty
  }
}
__global__ __launch_bounds__(kLedgerBlock) void k_ledger(DMesh m, DState s, DParams p, int nparts) {
  ledger_blk(m, s, p, nparts);
}

// mass (Neumaier-compensated), min and max of alpha: one block, fixed order
__global__ __launch_bounds__(1024) void k_stats(DMesh m, DState s, double *out) {
  __shared__ double rs[1024], rc[1024], rmn[1024], rmx[1024];
  double sum = 0.0, comp = 0.0, mn = 1e300, mx = -1e300;
  for (int64_t c = threadIdx.x; c < m.nc; c += 1024) {
    double a = s.alpha[c];
    double v = m.V[c] * a;
    double t = sum + v;
    comp += (fabs(sum) >= fabs(v)) ? (sum - t) + v : (v - t) + sum;
    sum = t;
    mn = dmin(mn, a);
    mx = dmax(mx, a);
  }
  rs[threadIdx.x] = sum; rc[threadIdx.x] = comp; rmn[threadIdx.x] = mn; rmx[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Cp = 0.0, lo = 1e300, hi = -1e300;
    for (int i = 0; i < 1024; ++i) {
      double v = rs[i];
      double t = S + v;
      Cp += (fabs(S) >= fabs(v)) ? (S - t) + v : (v - t) + S;
      S = t;
      Cp += rc[i];
      lo = dmin(lo, rmn[i]);
      hi = dmax(hi, rmx[i]);
    }
    out[0] = S + Cp;
    out[1] = lo;
    out[2] = hi;
    out[3] = 0.0;
  }
}

// Geometric mapping after a mesh change (Section 3, Algorithm 2): alpha of
// each cell c of the new mesh d from the reconstruction of the old mesh o.
// One old cell containing c: for an interface cell, the fill level of c under
// the old cell's plane, summed over the fan tetrahedra (c's centroid, face
// centre, consecutive face points) with the closed-form kept fraction; for
// any other class the old alpha.  Several old cells: c is their union, and
// gets the sum of alpha V over them.  A map entry out of range, or a cell
// with no entry or offsets outside [0, off[nc]], raises kFlagBadMap and
// writes NaN.
__global__ __launch_bounds__(kBlock) void k_map_alpha(DMesh d, double *alpha, const int32_t *off,
                                                      const int32_t *cells, DMesh o, DState os,
                                                      uint32_t *flags) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= d.nc) return;
  const int k0 = off[c], k1 = off[c + 1];
  bool bad = k0 < 0 || k1 <= k0 || k1 > off[d.nc];
  double a = NAN;
  if (!bad && k1 - k0 == 1) {
    const int oc = cells[k0];
    bad = oc < 0 || oc >= o.nc;
    if (!bad && os.cls[oc] != 1) {
      a = os.alpha[oc];
    } else if (!bad) {
      const double4 pl = os.plane[oc];
      const v3 n = xyz(pl), org = xyz(d.XC[c]);
      const double sn = pl.w - dot(n, org);
      double acc = 0.0, tot = 0.0;
      for (int k = d.cf_off[c]; k < d.cf_off[c + 1]; ++k) {
        const int sf = d.cf[k];
        const int f = sf >= 0 ? sf : ~sf;
        const double sg = sf >= 0 ? 1.0 : -1.0;
        const int b = d.foff[f], nn = d.foff[f + 1] - b;
        const v3 cf = xyz(d.C[f]) - org;
        const double hc = dot(n, cf);
        v3 pa = xyz(d.X[d.fpts[b + nn - 1]]) - org;
        for (int i = 0; i < nn; ++i) {
          const v3 pb = xyz(d.X[d.fpts[b + i]]) - org;
          const double v6 = sg * det3(cf, pa, pb);
          acc += v6 * tet_kept_fraction(D4{sn, sn - hc, sn - dot(n, pa), sn - dot(n, pb)});
          tot += v6;
          pa = pb;
        }
      }
      a = acc / tot;
    }
  } else if (!bad) {
    double v = 0.0;
    for (int k = k0; k < k1 && !bad; ++k) {
      const int oc = cells[k];
      bad = oc < 0 || oc >= o.nc;
      if (!bad) v += os.alpha[oc] * o.V[oc];
    }
    a = bad ? NAN : v / d.V[c];
  }
  if (bad) {
    a = NAN;
    flag(flags, kFlagBadMap);
  }
  alpha[c] = a;
}

// ---------------------------------------------------------------------------
// batches: one launch per kernel over the work of many meshes
// ---------------------------------------------------------------------------
// The mesh of global item g in an exclusive prefix `off` of n meshes (off[0]
// = 0, off[n] = the total, empty meshes repeat an offset): the i with
// off[i] <= g < off[i + 1].  Works on global or LDS arrays.
__device__ __forceinline__ int find_inst(const int32_t *off, int n, int g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Exclusive prefix over the batch's meshes of units(i) into pre[0..n] (LDS,
// kMaxBatch + 1 entries), and the mesh's count(i) into cnt[i]: every thread of
// the block takes a run of consecutive meshes, the runs' sums are scanned
// across the wave and then across the block's waves.  Whole block.
template <class Units>
__device__ void batch_prefix(int n, int32_t *pre, Units units) {
  __shared__ int32_t wtot[kBlock / kWave];
  const int T = (int)blockDim.x, W = T / kWave;
  const int per = (n + T - 1) / T;
  const int a = (int)threadIdx.x * per;
  int loc = 0;
  for (int k = 0; k < per; ++k)
    if (a + k < n) loc += units(a + k);
  const int lane = lane_id(), w = (int)threadIdx.x / kWave;
  int v = loc;
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == kWave - 1) wtot[w] = v;
  __syncthreads();
  int base = 0;
  for (int i = 0; i < w; ++i) base += wtot[i];
  int run = base + v - loc;
  for (int k = 0; k < per; ++k)
    if (a + k < n) {
      pre[a + k] = run;
      run += units(a + k);
    }
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < W; ++i) tot += wtot[i];
    pre[n] = tot;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void kb_begin(BTab t) {
  const int n = t.hdr[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    t.inst[i].s.stepno[0] = 0;
}

__global__ __launch_bounds__(kBlock) void kb_cell_class(BTab t) {
  const int n = t.hdr[0], tot = t.cls_off[n];
  for (int g = blockIdx.x; g < tot; g += gridDim.x) {
    const int i = find_inst(t.cls_off, n, g);
    const BInst &I = t.inst[i];
    cell_class_blk(I.m, I.s, I.p, g - t.cls_off[i], t.cls_off[i + 1] - t.cls_off[i]);
  }
}

__global__ __launch_bounds__(kBlock) void kb_point_prep(BTab t) {
  const int n = t.hdr[0], tot = t.pt_off[n];
  for (int g = blockIdx.x; g < tot; g += gridDim.x) {
    const int i = find_inst(t.pt_off, n, g);
    const BInst &I = t.inst[i];
    point_prep_one(I.m, I.s, I.p, (int64_t)(g - t.pt_off[i]) * blockDim.x + threadIdx.x);
  }
}

// Interface cells of all meshes, four per wave at a time.
template <bool WIDE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void kb_plane(BTab t) {
  __shared__ int32_t pre[kMaxBatch + 1];
  const int n = t.hdr[0];
  batch_prefix(n, pre, [&](int i) { return (t.inst[i].s.work[kWInterface] + 3) / 4; });
  const int lane = lane_id();
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (int)((gridDim.x * blockDim.x) >> 6);
  unsigned long long nfall = 0;
  int cur = -1;
  for (int q = wave; q < pre[n]; q += nwaves) {
    const int i = find_inst(pre, n, q);
    if (i != cur) {
      if (cur >= 0) wave_count(cnt_at(t.inst[cur].s.cnt, kCntFallback), nfall);
      nfall = 0;
      cur = i;
    }
    const BInst &I = t.inst[i];
    plane_quad<WIDE>(I.m, I.s, I.p, q - pre[i], I.s.work[kWInterface], lane, nfall);
  }
  if (cur >= 0) wave_count(cnt_at(t.inst[cur].s.cnt, kCntFallback), nfall);
}

// Flux blocks of the meshes of one face kind; every XCD walks a contiguous
// range of the blocks (neighbouring faces share points, and so L2 lines).
template <int NMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NMAX <= 4 ? 4 : 1)))
void kb_flux(BTab t, int kind) {
  const int kn = t.hdr[1 + kind];
  const int32_t *list = t.klist + kind * kMaxBatch;
  const int32_t *off = t.kflux_off + kind * (kMaxBatch + 1);
  const int tot = off[kn];
  const int per = (int)gridDim.x / kXcds;  // blocks per XCD
  const int x = (int)blockIdx.x % kXcds, j = (int)blockIdx.x / kXcds;
  const int g0 = (int)((int64_t)tot * x / kXcds), g1 = (int)((int64_t)tot * (x + 1) / kXcds);
  unsigned long long nflux = 0, nit = 0, nbad = 0;
  int cur = -1;
  for (int g = g0 + j; g < g1; g += per) {
    const int k = find_inst(off, kn, g);
    if (k != cur) {
      if (cur >= 0) {
        const DState &S = t.inst[list[cur]].s;
        block_count3(cnt_at(S.cnt, kCntFaceFluxes), nflux, cnt_at(S.cnt, kCntIters), nit,
                     cnt_at(S.cnt, kCntUnreached), nbad);
        __syncthreads();
      }
      nflux = nit = nbad = 0;
      cur = k;
    }
    const BInst &I = t.inst[list[k]];
    const int step = *I.s.stepno;
    flux_chunk<NMAX>(I.m, I.s, I.p, (int64_t)(g - off[k]) * blockDim.x, I.s.dt[step],
                     I.s.sc[step], nflux, nit, nbad);
  }
  if (cur >= 0) {
    const DState &S = t.inst[list[cur]].s;
    block_count3(cnt_at(S.cnt, kCntFaceFluxes), nflux, cnt_at(S.cnt, kCntIters), nit,
                 cnt_at(S.cnt, kCntUnreached), nbad);
  }
}

// Face groups of the geometric faces of the meshes of one face kind, claimed
// `claim` at a time (the first by block index, the rest from a counter).
// Prefix of the face groups of the register clip over the meshes of each
// face kind (one block; after the flux kernels): kept in global memory, as
// the clip kernel's LDS is what bounds its occupancy.
__global__ __launch_bounds__(kBlock) void kb_group_prefix(BTab t) {
  __shared__ int32_t pre[kMaxBatch + 1];
  for (int kind = 0; kind < kFaceKinds; ++kind) {
    const int kn = t.hdr[1 + kind];
    const int32_t *list = t.klist + kind * kMaxBatch;
    batch_prefix(kn, pre, [&](int k) {
      const BInst &I = t.inst[list[k]];
      return clip_groups(I.m, I.s).total;
    });
    for (int k = threadIdx.x; k <= kn; k += blockDim.x)
      t.gpre[kind * (kMaxBatch + 1) + k] = pre[k];
    __syncthreads();
  }
}

template <int SLOTS, int CAND, bool BOXES, int MAXPL, bool CHUNKED>
__global__ __launch_bounds__(kFastBlock) __attribute__((amdgpu_waves_per_eu(BOXES ? 3 : 2)))
void kb_clip_fast(BTab t, int kind, int claim) {
  __shared__ int group;
  const int kn = t.hdr[1 + kind];
  const int32_t *list = t.klist + kind * kMaxBatch;
  const int32_t *pre = t.gpre + kind * (kMaxBatch + 1);
  const int lane = threadIdx.x;
  const int ngroups = pre[kn];
  unsigned long long npairs = 0, nresc = 0;
  int cur = -1, left = -1;
  for (;;) {
    if (lane == 0) {
      if (left < 0) {
        group = claim * (int)blockIdx.x;
        left = claim;
      } else if (left == 0) {
        group = claim * ((int)gridDim.x + atomicAdd(&t.work[kBWClip + kind], 1));
        left = claim;
      } else {
        group = group + 1;
      }
      --left;
    }
    __syncthreads();
    const int g = group;
    if (g >= ngroups) break;
    const int k = find_inst(pre, kn, g);
    if (k != cur) {
      if (cur >= 0) {
        const DState &S = t.inst[list[cur]].s;
        wave_count(cnt_at(S.cnt, kCntPairs), npairs);
        wave_count(cnt_at(S.cnt, kCntRescans), nresc);
      }
      npairs = nresc = 0;
      cur = k;
    }
    const BInst &I = t.inst[list[k]];
    const int step = *I.s.stepno;
    const double sweep = -I.s.sc[step] * I.s.dt[step];
    const ClipGroups cg = clip_groups(I.m, I.s);
    const int gl = g - pre[k];
    const bool sm = gl < cg.nsmall;
    clip_fast_group<SLOTS, CAND, BOXES, MAXPL, CHUNKED>(
        I.m, I.s, I.p, sm ? gl : gl - cg.nsmall, sm ? cg.na : cg.nb, sm ? 0 : (int)I.m.nf - 1,
        sm ? 1 : -1, sm ? cg.tsmall : I.m.tpf, sweep, npairs, nresc);
  }
  if (cur >= 0) {
    const DState &S = t.inst[list[cur]].s;
    wave_count(cnt_at(S.cnt, kCntPairs), npairs);
    wave_count(cnt_at(S.cnt, kCntRescans), nresc);
  }
}

__global__ __launch_bounds__(kClipBlock) __attribute__((amdgpu_waves_per_eu(2))) void kb_clip_general(BTab t) {
  __shared__ int32_t pre[kMaxBatch + 1];
  const int n = t.hdr[0];
  batch_prefix(n, pre, [&](int i) {
    return (t.inst[i].s.work[kWDeferred] + kGenTets - 1) / kGenTets;
  });
  unsigned long long ncap = 0, npairs = 0;
  int cur = -1;
  for (int q = blockIdx.x; q < pre[n]; q += gridDim.x) {
    const int i = find_inst(pre, n, q);
    if (i != cur) {
      if (cur >= 0) clip_general_counts(t.inst[cur].s, ncap, npairs);
      ncap = npairs = 0;
      cur = i;
    }
    const BInst &I = t.inst[i];
    const int step = *I.s.stepno;
    clip_general_tets(I.m, I.s, I.p, (q - pre[i]) * kGenTets, I.s.work[kWDeferred],
                      I.s.dt[step], I.s.sc[step], ncap, npairs);
  }
  if (cur >= 0) clip_general_counts(t.inst[cur].s, ncap, npairs);
}

__global__ __launch_bounds__(kBlock) void kb_face_sum(BTab t) {
  __shared__ int32_t pre[kMaxBatch + 1];
  const int n = t.hdr[0];
  batch_prefix(n, pre, [&](int i) {
    return (geo_count(t.inst[i].s) + kBlock - 1) / kBlock;
  });
  unsigned long long nleak = 0;
  int cur = -1;
  for (int q = blockIdx.x; q < pre[n]; q += gridDim.x) {
    const int i = find_inst(pre, n, q);
    if (i != cur) {
      if (cur >= 0) face_sum_counts(t.inst[cur].s, nleak);
      nleak = 0;
      cur = i;
    }
    const BInst &I = t.inst[i];
    const int f = (q - pre[i]) * kBlock + (int)threadIdx.x;
    if (f < geo_count(I.s)) face_sum_one(I.m, I.s, I.p, f, I.s.work[kWGeometric], nleak);
  }
  if (cur >= 0) face_sum_counts(t.inst[cur].s, nleak);
}

__global__ __launch_bounds__(kBlock) void kb_update(BTab t) {
  const int n = t.hdr[0], tot = t.upd_off[n];
  for (int g = blockIdx.x; g < tot; g += gridDim.x) {
    const int i = find_inst(t.upd_off, n, g);
    const BInst &I = t.inst[i];
    update_blk(I.m, I.s, I.p, g - t.upd_off[i]);
  }
}

// one block per mesh; the first block also clears the batch's claim counters
__global__ __launch_bounds__(kLedgerBlock) void kb_ledger(BTab t) {
  const int n = t.hdr[0];
  if (blockIdx.x == 0 && threadIdx.x < kBWNum) t.work[threadIdx.x] = 0;
  if ((int)blockIdx.x >= n) return;
  const BInst &I = t.inst[blockIdx.x];
  ledger_blk(I.m, I.s, I.p, (int)grid_for_dev(I.m.nc, kBlock));
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_mesh_geometry(const DMesh &m0, double4 *X, const double *pts, double4 *S, double4 *C,
                          double *V, double4 *XC, double *wpc, double4 *cpl, uint8_t *npl,
                          uint8_t *isbox, uint8_t *fan_w, double4 *bblo,
                          double4 *bbhi, uint32_t *flags, hipStream_t st) {
  DMesh m = m0;
  k_points<<<grid_for(m.np, kBlock), kBlock, 0, st>>>(m.np, pts, X);
  k_face_geom<<<grid_for(m.nf, kBlock), kBlock, 0, st>>>(m, S, C);
  k_cell_geom<<<grid_for(m.nc, kBlock), kBlock, 0, st>>>(m, V, XC, bblo, bbhi);
  k_cell_planes<<<grid_for(m.nc, kBlock), kBlock, 0, st>>>(m, cpl, npl, isbox, fan_w, bblo,
                                                            bbhi);
  k_idw<<<grid_for(m.np, kBlock), kBlock, 0, st>>>(m, wpc);
  if (m.ni > 0) k_check_orientation<<<grid_for(m.ni, kBlock), kBlock, 0, st>>>(m, flags);
}

void launch_point_velocity(const DMesh &m, const double *U0c, double4 *U, double *XU, double *coef,
                           hipStream_t st) {
  k_point_velocity<<<grid_for(m.np, kBlock), kBlock, 0, st>>>(m, U0c, U, XU);
  if (m.maxn <= 3)
    k_face_coeffs<3><<<grid_for(m.nf, kBlock), kBlock, 0, st>>>(m, XU, coef);
  else if (m.maxn == 4)
    k_face_coeffs<4><<<grid_for(m.nf, kBlock), kBlock, 0, st>>>(m, XU, coef);
  else
    k_face_coeffs<kMaxFacePoints><<<grid_for(m.nf, kBlock), kBlock, 0, st>>>(m, XU, coef);
}

static void launch_plane(const DMesh &m, const DState &s, const DParams &p, hipStream_t st) {
  if (m.wide)
    k_plane<true><<<kPlaneGrid, kBlock, 0, st>>>(m, s, p);
  else
    k_plane<false><<<kPlaneGrid, kBlock, 0, st>>>(m, s, p);
}

static void launch_reconstruct_impl(const DMesh &m, const DState &s, const DParams &p,
                                    hipStream_t st) {
  k_cell_class<<<grid_for(m.nc, kBlock * kClassCells), kBlock, 0, st>>>(m, s, p);
  k_point_prep<<<grid_for(m.np, kBlock), kBlock, 0, st>>>(m, s, p);
  launch_plane(m, s, p, st);
}

// A step starts from zero work counters (the previous step's last kernel
// clears them), so a reconstruction clears them again when it is done.
void launch_reconstruct(const DMesh &m, const DState &s, const DParams &p, hipStream_t st) {
  k_reset<<<1, 64, 0, st>>>(s);
  launch_reconstruct_impl(m, s, p, st);
  k_reset<<<1, 64, 0, st>>>(s);
}

bool Prof::begin(int kid) {
  if (n >= cap) return false;
  (void)hipEventRecord(recs[n].a, st);
  recs[n].kid = kid;
  return true;
}
void Prof::end(int kid) {
  (void)kid;
  (void)hipEventRecord(recs[n].b, st);
  ++n;
}

// kernel launch bracketed by timing events when profiling
#define TIMED(prof, kid, launch)                       \
  do {                                                 \
    bool on_ = (prof) && (prof)->begin(kid);           \
    launch;                                            \
    if (on_) (prof)->end(kid);                         \
  } while (0)

// One step of the path; the step index (for dt and scale) is read by the
// kernels from s.stepno, which the last kernel advances, so the same launch
// sequence serves every step (and is captured once as a graph).  The flux
// kernel needs the point masks but not the planes, so with a Fork the plane
// kernel runs beside it.
void launch_step(const DMesh &m, const DState &s, const DParams &p, hipStream_t st, Prof *prof,
                 const Fork *fork) {
  const bool split = fork && !prof;
  TIMED(prof, kKCellClass,
        (k_cell_class<<<grid_for(m.nc, kBlock * kClassCells), kBlock, 0, st>>>(m, s, p)));
  TIMED(prof, kKPointPrep, (k_point_prep<<<grid_for(m.np, kBlock), kBlock, 0, st>>>(m, s, p)));
  if (split) {
    (void)hipEventRecord(fork->fork, st);
    (void)hipStreamWaitEvent(fork->side, fork->fork, 0);
    launch_plane(m, s, p, fork->side);
    (void)hipEventRecord(fork->join, fork->side);
  } else {
    TIMED(prof, kKPlane, launch_plane(m, s, p, st));
  }
  // persistent-style grid, a multiple of the XCD count
  unsigned gf = grid_for(m.nf, kBlock);
  gf = gf < kFluxGrid ? gf : kFluxGrid;
  gf = (gf + kXcds - 1) / kXcds * kXcds;
  if (m.maxn <= 3)
    TIMED(prof, kKFlux, (k_flux<3><<<gf, kBlock, 0, st>>>(m, s, p)));
  else if (m.maxn == 4)
    TIMED(prof, kKFlux, (k_flux<4><<<gf, kBlock, 0, st>>>(m, s, p)));
  else
    TIMED(prof, kKFlux, (k_flux<kMaxFacePoints><<<gf, kBlock, 0, st>>>(m, s, p)));
  if (split) (void)hipStreamWaitEvent(st, fork->join, 0);
  if (m.maxn <= 3)
    TIMED(prof, kKClip,
          (k_clip_fast<kTriSlots, kTriCand, false, kTriPlanes, true>
           <<<kFastGrid, kFastBlock, 0, st>>>(m, s, p)));
  else
    TIMED(prof, kKClip,
          (k_clip_fast<kFastSlots, kCandPool, true, kFastPlanes, false>
           <<<kFastGrid, kFastBlock, 0, st>>>(m, s, p)));
  TIMED(prof, kKClipGeneral, (k_clip_general<<<4096, kClipBlock, 0, st>>>(m, s, p)));
  TIMED(prof, kKFaceSum, (k_face_sum<<<1024, kBlock, 0, st>>>(m, s, p)));
  TIMED(prof, kKUpdate, (k_update<<<grid_for(m.nc, kBlock), kBlock, 0, st>>>(m, s, p)));
  if (p.wisps)
    TIMED(prof, kKWisps, (k_wisp_receivers<<<kWispGrid, kBlock, 0, st>>>(m, s, p),
                          k_wisp_offers<<<kWispGrid, kBlock, 0, st>>>(m, s, p),
                          k_wisp_sums<<<kWispGrid, kBlock, 0, st>>>(m, s, p),
                          k_wisp_moves<<<kWispGrid, kBlock, 0, st>>>(m, s, p)));
  TIMED(prof, kKLedger,
        (k_ledger<<<1, kLedgerBlock, 0, st>>>(m, s, p, (int)grid_for(m.nc, kBlock))));
}

void launch_batch_begin(const BTab &t, int n, hipStream_t st) {
  if (n > 0) kb_begin<<<grid_for(n, kBlock), kBlock, 0, st>>>(t);
}

// One step of a batch: the single-mesh step's kernels, each over all meshes
// (the flux and register-clip kernels once per face kind present).
void launch_batch_step(const BTab &t, const BConf &c, unsigned kinds, int ledger_grid,
                       hipStream_t st, const Fork *fork, hipEvent_t *ev) {
  // ev (eager launches only): 0 start, 1 after the cell and point kernels, 2 after
  // the plane kernel, 3 after the flux kernels, 4 after the register clips,
  // 5 before the update, 6 after the update, 7 after the ledger
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], st);
  };
  mark(0);
  kb_cell_class<<<c.grid_cells, kBlock, 0, st>>>(t);
  kb_point_prep<<<c.grid_cells, kBlock, 0, st>>>(t);
  mark(1);
  if (fork && !ev) {
    (void)hipEventRecord(fork->fork, st);
    (void)hipStreamWaitEvent(fork->side, fork->fork, 0);
    if (kinds & 8u)
      kb_plane<true><<<c.grid_plane, kBlock, 0, fork->side>>>(t);
    else
      kb_plane<false><<<c.grid_plane, kBlock, 0, fork->side>>>(t);
    (void)hipEventRecord(fork->join, fork->side);
  } else {
    if (kinds & 8u)
      kb_plane<true><<<c.grid_plane, kBlock, 0, st>>>(t);
    else
      kb_plane<false><<<c.grid_plane, kBlock, 0, st>>>(t);
  }
  mark(2);
  const int gf = (c.grid_flux + kXcds - 1) / kXcds * kXcds;
  if (kinds & 1u) kb_flux<3><<<gf, kBlock, 0, st>>>(t, 0);
  if (kinds & 2u) kb_flux<4><<<gf, kBlock, 0, st>>>(t, 1);
  if (kinds & 4u) kb_flux<kMaxFacePoints><<<gf, kBlock, 0, st>>>(t, 2);
  if (fork && !ev) (void)hipStreamWaitEvent(st, fork->join, 0);
  mark(3);
  kb_group_prefix<<<1, kBlock, 0, st>>>(t);
  if (kinds & 1u)
    kb_clip_fast<kTriSlots, kTriCand, false, kTriPlanes, true>
        <<<c.grid_clip, kFastBlock, 0, st>>>(t, 0, c.clip_claim);
  if (kinds & 2u)
    kb_clip_fast<kFastSlots, kCandPool, true, kFastPlanes, false>
        <<<c.grid_clip, kFastBlock, 0, st>>>(t, 1, c.clip_claim);
  if (kinds & 4u)
    kb_clip_fast<kFastSlots, kCandPool, true, kFastPlanes, false>
        <<<c.grid_clip, kFastBlock, 0, st>>>(t, 2, c.clip_claim);
  mark(4);
  kb_clip_general<<<4096, kClipBlock, 0, st>>>(t);
  kb_face_sum<<<1024, kBlock, 0, st>>>(t);
  mark(5);
  kb_update<<<c.grid_cells, kBlock, 0, st>>>(t);
  mark(6);
  kb_ledger<<<ledger_grid, kLedgerBlock, 0, st>>>(t);
  mark(7);
}

void launch_map_alpha(const DMesh &d, double *alpha, const int32_t *off, const int32_t *cells,
                      const DMesh &o, const DState &os, uint32_t *flags, hipStream_t st) {
  if (d.nc > 0)
    k_map_alpha<<<grid_for(d.nc, kBlock), kBlock, 0, st>>>(d, alpha, off, cells, o, os, flags);
}

void launch_stats(const DMesh &m, const DState &s, double *out4, hipStream_t st) {
  k_stats<<<1, 1024, 0, st>>>(m, s, out4);
}

// Host evaluation of the same clipping code (self-test, no GPU needed).
double host_tet_clip(const double *tet, int n_planes, const double *planes) {
  double px[kPolyCap], py[kPolyCap], pz[kPolyCap], ps[kPolyCap];
  uint8_t nb[3 * kPolyCap], aux[kPolyCap];
  Poly P;
  P.px = px; P.py = py; P.pz = pz; P.ps = ps; P.nb = nb; P.aux = aux;
  P.st = 1; P.cap = kPolyCap; P.nv = 0;
  v3 a = mk3(tet[0], tet[1], tet[2]), b = mk3(tet[3], tet[4], tet[5]);
  v3 c = mk3(tet[6], tet[7], tet[8]), d = mk3(tet[9], tet[10], tet[11]);
  if (det3(b - a, c - a, d - a) < 0.0) { v3 t = c; c = d; d = t; }
  P.init_tet(a, b, c, d);
  for (int k = 0; k < n_planes; ++k)
    if (!P.clip(mk3(planes[4 * k], planes[4 * k + 1], planes[4 * k + 2]), planes[4 * k + 3]))
      return NAN;
  return P.vol6() / 6.0;
}

// Host evaluation of the register-only closed forms, with the tetrahedron
// moved so that its first vertex is the origin as in the clip kernels.
double host_tet_clip_closed(const double *tet, int n_planes, const double *planes) {
  if (n_planes > kRegPlanes) return NAN;
  v3 a = mk3(tet[0], tet[1], tet[2]), b = mk3(tet[3], tet[4], tet[5]);
  v3 c = mk3(tet[6], tet[7], tet[8]), d = mk3(tet[9], tet[10], tet[11]);
  if (det3(b - a, c - a, d - a) < 0.0) { v3 t = c; c = d; d = t; }
  const Tet T{mk3(0, 0, 0), b - a, c - a, d - a};
  Pl pl[kRegPlanes] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int k = 0; k < n_planes; ++k) {
    v3 n = mk3(planes[4 * k], planes[4 * k + 1], planes[4 * k + 2]);
    pl[k] = mkpl(n, planes[4 * k + 3] - dot(n, a));
  }
  const double det = det3(T.b, T.c, T.d);
  const double one = vol6_planes(T, det, pl[0], pl[1], pl[2], pl[3], n_planes);
  if (n_planes < 2) return one / 6.0;
  // the split terms as the three lanes of a queued pair add them
  double t[3];
  for (int i = 0; i < 3; ++i)
    t[i] = n_planes == 2   ? split_term<2>(dist_table<2>(T, pl[0], pl[1], pl[2], pl[3]), i)
           : n_planes == 3 ? split_term<3>(dist_table<3>(T, pl[0], pl[1], pl[2], pl[3]), i)
                           : split_term<4>(dist_table<4>(T, pl[0], pl[1], pl[2], pl[3]), i);
  const double three = det * ((t[0] + t[1]) + t[2]);
  if (!(fabs(three - one) <= 1e-14 * det)) return NAN;
  return three / 6.0;
}

}  // namespace vof
