// vof_internal.h -- device-side data layout of the flux library (internal).
//
// Layout in HBM.  Gathered per-point data are 32-byte double4 records so one
// aligned load brings a whole point (coordinates, or velocity); everything
// streamed per face or per cell is a plain array indexed by face or cell.
// CSR addressing (int32 offsets) for face -> points, cell -> faces (signed:
// f for an owned face, ~f for a neighbour face, eq. 2.5), point -> cells and
// face -> stencil cells.  Cell planes are stored per cell -> face entry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vof {

constexpr int kMaxFacePoints = 8;   // points of one face
constexpr int kPolyCap = 24;        // vertices of one clipped polytope
constexpr int kMaxCellPlanes = 16;  // planes of one cell tested per tet
// Geometric faces of a step come in two lists in gfaces: faces of up to
// kSmallFace points from its front (work[kWGeometric] of them), faces of
// more points from its end (work[kWGeoLarge]).  The register clip takes each
// list in groups of its own width (5 tets per face point), so the few larger
// faces of a refined mesh (hanging nodes) do not widen the groups of all its
// other faces.  Tet storage keeps the mesh's stride of 5 * maxn per slot.
constexpr int kSmallFace = 4;

// status bits latched on the device
constexpr uint32_t kFlagCapacity = 1u;
constexpr uint32_t kFlagUnreached = 2u;
constexpr uint32_t kFlagNonFinite = 4u;
constexpr uint32_t kFlagLeak = 8u;
constexpr uint32_t kFlagBadOrientation = 16u;
constexpr uint32_t kFlagBadMap = 32u;

// 64-bit counters accumulated across steps
enum Counter : int {
  kCntSteps = 0,
  kCntFaceFluxes,
  kCntGeometric,
  kCntInterface,
  kCntFallback,
  kCntUnreached,
  kCntCapacity,
  kCntLeaks,
  kCntIters,
  kCntPairs,
  kCntDeferred,
  kCntWisps,
  kCntWispsLeft,
  kCntRescans,
  kCntNum
};

// per-step work counters (reset every step)
// Each counter is spread over kCntLanes slots, one 128-byte line apart,
// picked by block index: atomics of many blocks on one address serialise in
// L2.  The host adds the slots when it reads the counters.
constexpr int kCntLanes = 64;
constexpr int kCntStride = 16;
constexpr int64_t kCntWords = (int64_t)kCntNum * kCntLanes * kCntStride;

enum WorkCounter : int {
  kWInterface = 0, kWGeometric = 1, kWDeferred = 2, kWClipNext = 3, kWWisps = 4, kWRecv = 5,
  kWGeoLarge = 6, kWNum = 7
};

struct DMesh {
  int64_t np, nc, nf, ni;
  int32_t maxn;    // max points per face
  int32_t tpf;     // tetrahedra per face slot (5 * maxn)
  int32_t wide;    // 1: some cell has more than 64 face-fan tetrahedra (a whole wave in the
                   // plane kernel)
  const double4 *X;        // points (x, y, z, 0)
  const int32_t *foff;     // nf + 1
  const int32_t *fpts;     // face points
  const int32_t *fpad;     // face points padded to padw per face (-1 past the last)
  int32_t padw;            // 4 when every face has at most 4 points, else 8
  const int32_t *own;      // nf
  const int32_t *nei;      // ni
  const int32_t *cf_off;   // nc + 1
  const int32_t *cf;       // signed face index
  const int32_t *pc_off;   // np + 1
  const int32_t *pc;       // point -> cells
  const double *wpc;       // inverse distance weights (eq. 2.7)
  const int32_t *cpn_off;  // nc + 1: cells sharing a point with the cell (built on
  const int32_t *cpn;      // first use of the least-squares gradient), sorted
  const int32_t *st_off;   // nf + 1
  const int32_t *st;       // face -> stencil cells
  const double4 *S;        // face area vector, w = |S|
  const double4 *C;        // face centre (mean of points)
  const double *V;         // cell volume
  const double4 *XC;       // cell centroid
  const double4 *cpl;      // per cell, from cf_off[c]: its distinct face planes
                           // (outward unit normal, offset), npl[c] of them
  const uint8_t *npl;
  const uint8_t *isbox;    // 1: the cell is its bounding box (six axis planes at its bounds)
  const uint8_t *fan_w;      // lanes of the cell's plane group: 16 (at most 16 faces and 32
                             // face-fan tetrahedra), 32 (32 and 64) or 64
  const double4 *bblo;     // cell bounding box
  const double4 *bbhi;
};

struct DParams {
  double eps;
  double corr_rtol;
  int32_t corr_max_iter;
  double pos_tol;
  int32_t pos_max_iter;
  double grad_zero;
  int32_t check_stencil;
  int32_t gradient;        // 0 NAG, 1 generalized least squares
  int32_t band;            // bulk cells are not updated
  int32_t wisps;           // wisp redistribution after the update
};

struct DState {
  double *alpha;        // nc
  int8_t *cls;          // nc: 0 empty, 1 interface, 2 full, 3 vanishing gradient
  double4 *plane;       // nc: unit normal, s  (phase: n.x <= s)
  uint8_t *pmask;       // np: bit 1 empty, 2 full, 4 interface among point-cells
  double *alpha_p;      // np: IDW point values (band points only)
  double4 *U;           // np: reference point velocity
  double *XU;           // 6 np: position and reference velocity of each point, adjacent
                        // (48 bytes, three 16-byte loads)
  double *F0;           // nf
  double *coef;         // 3 nf: the volume cubic of each face for a unit sweep factor
                        // (C1, C2, C3 as three arrays of nf), set with the velocity
  double *lam;          // nf
  double *vphase;       // nf
  double *vscale;       // nf: F dt / V(lam) of a clamped face whose polyhedron holds at
                        // least a quarter of F dt (its phase fraction is scaled to F dt)
  uint8_t *iters;       // nf
  uint8_t *kind;        // nf
  uint8_t *fstatus;     // nf
  int32_t *icells;      // interface cell list
  int32_t *gfaces;      // geometric faces: up to kSmallFace points from the front, more from the end
  double *tetvol;       // per geometric face slot x tet
  double *tetdef;       // stencil check only: uncovered signed tet volume
  double *tetgross;     // stencil check only: unsigned tet volume
  int32_t *defer;       // flux tets left to the general clipper
  int32_t *work;        // per-step counters (kWNum)
  unsigned long long *cnt;  // kCntWords (kCntNum counters x kCntLanes slots)
  uint32_t *flags;      // latched status bits
  double *ledger;       // accumulated boundary phase volume
  double *part;         // per update block: its cells' boundary phase volume
  int32_t *stepno;      // index into dt / sc of the step being run
  double *dt;           // per-step dt (device copy)
  double *sc;           // per-step scale
  // narrow band
  uint8_t *inexact;     // nc: class empty or full but alpha not exactly 0 or 1
  uint8_t *fbulk;       // nf: 1 (2) when every point-cell of every face point is exactly 0 (1)
  // wisp redistribution (cells stamped with the running step's stamp are
  // this step's wisps or receivers; stamps start at 1, arrays at 0)
  uint32_t *wctr;       // stamp of the last finished step
  uint32_t *wstamp;     // nc
  uint32_t *rstamp;     // nc
  int32_t *wlist;       // wisps of this step
  int32_t *rlist;       // receivers of this step
  double *wex;          // nc: signed excess volume (alpha - target) V of a wisp
  double *wsum;         // nc: per wisp, sum of its receivers' offer ratios
  double2 *rho;         // nc: per receiver, room / sum of m > 0, store / sum of -m, m < 0
};

// Batches: many meshes advanced by the same launches.  Every mesh keeps its
// own addressing and state; a device table holds their descriptors, and each
// batch kernel walks a work space spanning all of them (blocks, wave items or
// face groups of one mesh at a time), running the single-mesh kernels' code
// on that mesh's descriptors.  Meshes are grouped by face kind for the
// kernels whose code depends on the number of points per face.
constexpr int kMaxBatch = 256;
constexpr int kFaceKinds = 3;  // 0: at most 3 points per face, 1: 4, 2: 5..8
inline int face_kind(int maxn) { return maxn <= 3 ? 0 : (maxn == 4 ? 1 : 2); }
enum BatchWork : int { kBWClip = 0, kBWNum = kBWClip + kFaceKinds };
struct BInst {
  DMesh m;
  DState s;   // the mesh's state, with dt / sc pointing at the batch's schedule
  DParams p;
};
struct BTab {
  const int32_t *hdr;        // [0] meshes n, [1 + k] meshes of face kind k
  const BInst *inst;         // n
  const int32_t *cls_off;    // n + 1: prefix of cell-class blocks (kBlock * 8 cells)
  const int32_t *pt_off;     // n + 1: prefix of point blocks (kBlock points)
  const int32_t *upd_off;    // n + 1: prefix of update blocks (kBlock cells)
  const int32_t *klist;      // kFaceKinds x kMaxBatch: the meshes of each face kind
  const int32_t *kflux_off;  // kFaceKinds x (kMaxBatch + 1): prefix of flux blocks over klist
  int32_t *gpre;             // kFaceKinds x (kMaxBatch + 1): prefix of register-clip face
                             // groups over klist (written each step)
  int32_t *work;             // kBWNum claim counters (cleared by the ledger)
};
// launch configuration of a batch step (what the autotuner picks)
struct BConf {
  int grid_flux;     // persistent blocks of the flux kernel (multiple of 8)
  int grid_clip;     // waves of the register clip
  int clip_claim;    // face groups taken per claim
  int grid_plane;    // blocks of four waves for the plane kernel
  int grid_cells;    // blocks of the cell and point kernels
};

// Per-kernel timing with HIP events on the launch stream (optional).
enum KernelId : int {
  kKReset = 0, kKCellClass, kKPointPrep, kKPlane, kKFlux, kKClip, kKClipGeneral, kKFaceSum,
  kKUpdate, kKLedger, kKWisps, kKNum
};
struct Prof {
  struct Rec { int kid; hipEvent_t a, b; };
  Rec *recs = nullptr;  // pool of recorded pairs
  int n = 0, cap = 0;
  hipStream_t st = nullptr;
  bool begin(int kid);  // records the start event; false if the pool is full
  void end(int kid);
};

// launchers (vof_device.hip)
void launch_mesh_geometry(const DMesh &m, double4 *X, const double *pts, double4 *S, double4 *C,
                          double *V, double4 *XC, double *wpc, double4 *cpl, uint8_t *npl,
                          uint8_t *isbox, uint8_t *fan_w, double4 *bblo,
                          double4 *bbhi, uint32_t *flags, hipStream_t st);
void launch_point_velocity(const DMesh &m, const double *U0c, double4 *U, double *XU, double *coef,
                           hipStream_t st);
// A second stream and two events: when given (and not profiling), the PLIC
// planes are computed on `side` while the flux kernel runs on the main stream
// (neither reads what the other writes); the clip waits for both.
struct Fork {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
void launch_step(const DMesh &m, const DState &s, const DParams &p, hipStream_t st, Prof *prof,
                 const Fork *fork);
void launch_reconstruct(const DMesh &m, const DState &s, const DParams &p, hipStream_t st);
void launch_stats(const DMesh &m, const DState &s, double *out4, hipStream_t st);
void launch_map_alpha(const DMesh &d, double *alpha, const int32_t *off, const int32_t *cells,
                      const DMesh &o, const DState &os, uint32_t *flags, hipStream_t st);
// One batch step on `st` (plane kernel on fork->side when given).  `kinds`
// bit k: some mesh has face kind k (launches for absent kinds are skipped);
// `ledger_grid`: blocks of the ledger (at least the number of meshes).
// ev: NULL, or 8 events recorded between the kernel groups (eager launch on
// `st` only; the fork is then not used).
void launch_batch_step(const BTab &t, const BConf &c, unsigned kinds, int ledger_grid,
                       hipStream_t st, const Fork *fork, hipEvent_t *ev = nullptr);
// Set every mesh's step counter to 0 (before a batch's first step).
void launch_batch_begin(const BTab &t, int n, hipStream_t st);
double host_tet_clip(const double *tet, int n_planes, const double *planes);
double host_tet_clip_closed(const double *tet, int n_planes, const double *planes);

}  // namespace vof
