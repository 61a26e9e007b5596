/*
 * vof.h -- C ABI of the MI355X geometric PLIC VoF flux library.
 *
 * The library advances a volume fraction field alpha on an unstructured
 * finite-volume mesh with the geometric, directionally unsplit PLIC method of
 * Maric, Marschall & Bothe (arXiv:1305.3417, "voFoam"), Section 2.  One time
 * step is the five-part path:
 *
 *   1. backtrack every mesh point along its discrete Lagrangian trajectory
 *      x' = x - U_p dt (eq. 2.16), with U_p interpolated from cell velocities
 *      by inverse distance weighting (eqs. 2.6-2.7);
 *   2. build one flux polyhedron per face from the face and its swept image,
 *      its volume taken by tetrahedral decomposition (eqs. 2.18-2.19);
 *   3. correct each polyhedron iteratively, moving the swept end points along
 *      their trajectories until its signed volume equals F_f dt (eq. 2.17;
 *      Section 2.3), without topology changes;
 *   4. fit a PLIC plane in every interface cell (Algorithm 1: NAG gradient,
 *      eqs. 2.6-2.12, and iterative positioning, Section 2.2.2);
 *   5. intersect every flux polyhedron with the cells of its stencil and
 *      their PLIC half-spaces (eqs. 2.22-2.23) and apply the conservative
 *      update alpha_c -= (1/V_c) sum_f sgn_cf V_{f,alpha} (eqs. 2.2, 2.5).
 *
 * All arithmetic is IEEE double precision on the GPU.
 *
 * Conventions for every entry point:
 *  - Pointers are host or device pointers as stated by a `memory` argument
 *    (VOF_HOST or VOF_DEVICE).  The caller owns every buffer it passes; the
 *    library copies inputs before the call returns (host) or before the
 *    enqueued work that reads them completes (device: keep the buffer alive
 *    and unmodified until the next synchronising call).
 *  - Device work is enqueued on the context's HIP stream, in call order.
 *    vof_read_* and vof_get_stats synchronise that stream.
 *  - No C++ exception and no abort crosses this interface.  Every function
 *    returns a vof_status; on failure vof_last_error() describes it (a
 *    thread-local string valid until the next call on the same thread).
 *  - Device-side failures (polytope capacity overflow, stencil leaks when
 *    checked) are latched in a flag word on the device and reported by the
 *    next synchronising call.
 *  - One context per host thread; calls on the same mesh must not overlap.
 */
#ifndef VOF_H
#define VOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vof_status;

#define VOF_OK 0
#define VOF_EINVAL (-1)    /* bad argument                                      */
#define VOF_EBADMESH (-2)  /* mesh failed validation                            */
#define VOF_ENOMEM (-3)    /* device allocation failed                          */
#define VOF_EDEVICE (-4)   /* HIP runtime error; destroy the context             */
#define VOF_ENUMERIC (-5)  /* a non-finite value was produced                   */
#define VOF_ESTENCIL (-6)  /* a flux polyhedron left its stencil (leak check)   */
#define VOF_EBUSY (-7)     /* server: the job can never fit its budget, or the
                              queue is full                                      */
#define VOF_ECAPACITY (-8) /* a clipped polytope exceeded its vertex capacity   */

#define VOF_HOST 0
#define VOF_DEVICE 1

typedef struct vof_context vof_context;
typedef struct vof_mesh vof_mesh;

/* Create a context on HIP device `device`; all work goes on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  A mesh keeps a copy of the
 * device and stream of the context it was uploaded with, so the context may
 * be destroyed before its meshes; the stream must outlive every mesh. */
vof_status vof_context_create(int32_t device, void *hip_stream, vof_context **out);
vof_status vof_context_destroy(vof_context *ctx);
/* Thread-local description of the last failure on this thread. */
const char *vof_last_error(void);
/* Library version string. */
const char *vof_version(void);

/* Unstructured mesh in owner/neighbour face addressing (Section 2):
 * points are stored once; a face is an ordered list of point indices; the
 * owner of a face has the lower cell index; the right-hand rule on the
 * point order gives an area vector S_f pointing out of the owner into the
 * neighbour.  Internal faces (with a neighbour) come first: faces
 * [0, n_internal) are internal, [n_internal, n_faces) are boundary faces
 * whose S_f points out of the domain.  Cells must be convex with planar
 * faces; faces have 3..VOF_MAX_FACE_POINTS points. */
#define VOF_MAX_FACE_POINTS 8
typedef struct {
  int64_t n_points, n_cells, n_faces, n_internal;
  const double *points;        /* 3 * n_points, x y z interleaved          */
  const int64_t *face_offsets; /* n_faces + 1                              */
  const int32_t *face_points;  /* face_offsets[n_faces]                    */
  const int32_t *owner;        /* n_faces                                  */
  const int32_t *neighbour;    /* n_internal                               */
  int32_t memory;              /* VOF_HOST or VOF_DEVICE for all arrays    */
} vof_mesh_desc;

typedef struct {
  int64_t n_points, n_cells, n_faces, n_internal;
  int64_t stencil_entries;     /* sum over faces of the flux stencil size   */
  int32_t max_face_points;
  int32_t max_cell_faces;
  int64_t device_bytes;        /* device memory held by the mesh            */
} vof_mesh_info;

/* Validate the mesh on the host (index ranges, owner < neighbour, face
 * sizes), copy it to the device, and precompute the derived addressing and
 * geometry: cell -> faces with owner/neighbour signs (eq. 2.5), point ->
 * cells, face area vectors and centres, cell volumes and centroids,
 * inverse-distance weights (eq. 2.7), cell face planes, and the flux stencil
 * of every face (the cells of its points, Section 2.3).  Orientation of S_f
 * against the owner -> neighbour direction is checked on the device.
 * Errors: VOF_EINVAL, VOF_EBADMESH, VOF_ENOMEM, VOF_EDEVICE. */
vof_status vof_mesh_upload(vof_context *ctx, const vof_mesh_desc *desc, vof_mesh **out);
vof_status vof_mesh_destroy(vof_mesh *mesh);
vof_status vof_mesh_get_info(const vof_mesh *mesh, vof_mesh_info *out);

/* Method parameters.  Defaults: eps 1e-12 (interface band: eps < alpha <
 * 1 - eps; the paper's "reconstruction tolerance", Section 4.2),
 * correction_rtol 1e-15 (|V_f - F_f dt| <= rtol |F_f dt|), correction_max_iter
 * 50, position_tol 1e-15 (|fill level - alpha| at the plane),
 * position_max_iter 100, gradient_zero 1e-8 (|grad alpha| h_c below this makes
 * an interface cell homogeneous), check_stencil 0 (1: also clip every
 * flux tet against the empty cells of its stencil and flag any volume that
 * leaves the stencil), gradient VOF_GRADIENT_NAG (the interface normal from
 * the node-averaged Gauss gradient, eqs. 2.6-2.12; VOF_GRADIENT_LSQ: from the
 * generalized least-squares gradient over the cells sharing a point with the
 * cell, inverse-distance weighted, Section 2.2.1 -- the first reconstruction
 * with it builds that cell stencil on the host), narrow_band 0 (1: the narrow
 * band of Section 2.3 -- bulk cells, those whose cells sharing a point, the
 * cell included, all hold alpha exactly 0 or all exactly 1, are not updated;
 * their update is zero in exact arithmetic), wisps 0 (1: after every update,
 * wisps -- cells outside the interface band eps < alpha < 1 - eps whose
 * alpha is not exactly 0 or 1, over- and undershoots included -- move their
 * excess over 0 or 1 to the interface cells sharing a point with them
 * (Section 2.3): each receiver offers the room (1 - eps - alpha) V, or for a
 * deficit the store (alpha - eps) V, it has, shared among the wisps around
 * it in proportion to their excess; a wisp moves at most what it is offered,
 * split in proportion to the offers, and is set to exactly 0 or 1 when it
 * moves all of it.  No receiver leaves [eps, 1 - eps].  Needs the same cell
 * stencil as the least-squares gradient). */
#define VOF_GRADIENT_NAG 0
#define VOF_GRADIENT_LSQ 1
typedef struct {
  double eps;
  double correction_rtol;
  int32_t correction_max_iter;
  double position_tol;
  int32_t position_max_iter;
  double gradient_zero;
  int32_t check_stencil;
  int32_t gradient;
  int32_t narrow_band;
  int32_t wisps;
} vof_params;
vof_status vof_get_params(const vof_mesh *mesh, vof_params *out);
vof_status vof_set_params(vof_mesh *mesh, const vof_params *p);

/* Volume fraction state, n_cells doubles.  vof_set_alpha also clears the
 * stored PLIC planes (each positioning starts from the cell's previous plane,
 * Section 2.2.2), so that the results of a run depend only on its inputs,
 * and resets the statistics. */
vof_status vof_set_alpha(vof_mesh *mesh, const double *alpha, int32_t memory);
vof_status vof_read_alpha(vof_mesh *mesh, double *out, int32_t memory);

/* Geometric mapping of the volume fraction after a mesh change (Section 3,
 * Algorithm 2), e.g. after 2:1 refinement or its undoing.  src holds the old
 * mesh and its alpha; it is reconstructed (Algorithm 1, with src's
 * parameters), and every cell c of dst takes its alpha from the old cells
 * map_cells[map_offsets[c] .. map_offsets[c + 1] - 1]:
 *   - one old cell o that contains c (c refined from o, or the same cell):
 *     alpha_c = |C_c ∩ {n_o . x <= s_o}| / V_c for an interface cell o (the
 *     old plane intersected with the new cell), alpha_o for an empty, full or
 *     vanishing-gradient cell o;
 *   - several old cells whose union is c (c coarsened from them):
 *     alpha_c = sum_o alpha_o V_o / V_c.
 * Both meshes live on the same device.  map_offsets: n_cells(dst) + 1
 * int32 starting at 0, every cell with at least one entry; map_cells: int32
 * cells of src; both in `memory` (host arrays are checked before any work,
 * device arrays by the kernel).  Synchronises.  Clears dst's planes and
 * resets its statistics like vof_set_alpha.  Errors: VOF_EINVAL (null or equal meshes, different
 * devices, src alpha not set, a bad map -- then dst's alpha is not set),
 * VOF_ENOMEM, VOF_EDEVICE. */
vof_status vof_map_alpha(vof_mesh *dst, vof_mesh *src, const int32_t *map_offsets,
                         const int32_t *map_cells, int32_t memory);

/* Reference velocity: U0c (3 * n_cells, x y z interleaved, cell-centred) and
 * the reference face volumetric flux F0 (n_faces; discretely divergence
 * free, eq. 2.4).  Step n of vof_advect uses scale[n] * U0c and
 * scale[n] * F0.  The point velocities U0_p are interpolated here by inverse
 * distance weighting (eqs. 2.6-2.7), and each face's flux-polyhedron volume
 * cubic for a unit sweep (Section 2.3) is computed once. */
vof_status vof_set_velocity(vof_mesh *mesh, const double *U0c, const double *F0,
                            int32_t memory);

/* Step 4 alone on the current alpha: classify cells and fit the PLIC planes
 * of the interface cells (Algorithm 1).  Results via vof_read_planes.  Each
 * positioning starts from the cell's stored plane, so repeated calls agree
 * to the positioning tolerance, not bit for bit. */
vof_status vof_reconstruct(vof_mesh *mesh);

/* Advance alpha by n_steps explicit steps (steps 1-5 each); step n has length
 * dt[n] and velocity / flux scale scale[n].  dt and scale are host arrays of
 * n_steps doubles, copied before return.  Every step uses alpha^n for all of
 * its geometry (explicit Euler, eq. 2.2). */
vof_status vof_advect(vof_mesh *mesh, int32_t n_steps, const double *dt, const double *scale);

/* vof_advect for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same steps, bitwise the same results, with no allocation of any kind.  The
 * schedule (dt, scale: host arrays of n_steps doubles, copied before return)
 * is staged in a fixed buffer of the library on the mesh's device (room for
 * VOF_NOALLOC_MAX_STEPS steps, 1 MiB, held until the process ends) instead of
 * memory the mesh allocates, and the steps are launched kernel by kernel on
 * the mesh's stream (no graph is built, the per-kernel profile is not
 * recorded).  Every scratch array the kernels use otherwise was allocated
 * with the mesh.  The staging buffer is shared by every call on one device:
 * calls that overlap on one GPU (from several host threads, or on meshes with
 * different streams before the earlier call's steps have run) race on it.
 * Blocks until earlier work on the mesh's stream is done and the schedule is
 * staged.  Errors: VOF_EINVAL (n_steps < 0 or above VOF_NOALLOC_MAX_STEPS,
 * null or non-finite schedule, alpha or velocity not set), VOF_EDEVICE. */
#define VOF_NOALLOC_MAX_STEPS 65536
vof_status vof_advect_noalloc(vof_mesh *mesh, int32_t n_steps, const double *dt,
                              const double *scale);

/* Per-face results of the last step.  what: VOF_FACE_LAMBDA (double, the
 * corrected sweep factor), VOF_FACE_VPHASE (double, V_{f,alpha}, signed like
 * F_f), VOF_FACE_ITERS (uint8, correction iterations), VOF_FACE_KIND (uint8:
 * 0 no flux, 1 trivially empty stencil, 2 trivially full stencil,
 * 3 geometric, 4 correction target unreachable with a clamped polyhedron
 * under a quarter of F dt: the face carries the upwind (donor) cell's alpha
 * times F dt -- alpha of the owner for F > 0, of the neighbour for F < 0, 0
 * for inflow through a boundary face), VOF_FACE_STATUS (uint8: 0 ok, 1
 * correction target beyond the extremum of the swept volume on its monotone
 * branch through lambda = 0 (Section 2.3 does not treat it): lambda is set
 * to that extremum or to the plain sweep (+-1 on the same side), whichever is
 * nearer to 0; where the polyhedron there holds at least a quarter of F dt
 * (with its sign) its phase volume is scaled by F dt / V_f(lambda), the scalar
 * coefficient correction (kind 3), else the face takes the donor cell
 * (kind 4), unless its stencil is trivially empty or full). */
#define VOF_FACE_LAMBDA 0
#define VOF_FACE_VPHASE 1
#define VOF_FACE_ITERS 2
#define VOF_FACE_KIND 3
#define VOF_FACE_STATUS 4
vof_status vof_read_face(vof_mesh *mesh, int32_t what, void *out, int32_t memory);

/* Cell classes and planes of the last reconstruction: cls (int8, n_cells:
 * 0 empty, 1 interface, 2 full, 3 interface with vanishing gradient, treated
 * as homogeneous), normal (3 * n_cells doubles) and position s (n_cells) of
 * the plane n.x = s; the phase occupies n.x <= s.  Any pointer may be NULL. */
vof_status vof_read_planes(vof_mesh *mesh, int8_t *cls, double *normal, double *s,
                           int32_t memory);

/* Interpolated point velocities U0_p (3 * n_points doubles). */
vof_status vof_read_point_velocity(vof_mesh *mesh, double *out, int32_t memory);

typedef struct {
  int64_t steps;              /* steps advanced since vof_set_alpha         */
  int64_t face_fluxes;        /* sum over steps of faces with F_f != 0      */
  int64_t geometric_faces;    /* sum over steps of faces clipped            */
  int64_t interface_cells;    /* sum over steps of interface cells          */
  int64_t fallback_cells;     /* sum over steps of vanishing-gradient cells */
  int64_t unreached_faces;    /* corrections clamped at the branch extremum */
  int64_t capacity_overflows; /* clipped polytopes beyond capacity          */
  int64_t stencil_leaks;      /* flux tets leaving their stencil (if checked) */
  int64_t correction_iters;   /* sum of correction iterations               */
  int64_t clip_pairs;         /* (flux tet, stencil cell) pairs that overlap */
  int64_t general_tets;       /* flux tets clipped by the general polytope path */
  double ledger;              /* sum of V_{f,alpha} over boundary faces      */
  double mass;                /* sum_c V_c alpha_c (compensated)            */
  double alpha_min, alpha_max;
  int64_t wisps;              /* sum over steps of wisps found (wisps = 1)   */
  int64_t wisps_left;         /* of those, wisps with too little room around */
  int64_t chunk_rescans;      /* tetrahedral meshes: face groups whose stencils
                                 were scanned again for a further chunk of
                                 candidate cells (a face with more candidates
                                 than a group's share)                       */
} vof_stats;
/* Synchronises, computes mass and alpha range, and reports the counters.
 * Returns VOF_ECAPACITY / VOF_ESTENCIL if the corresponding counter is
 * non-zero (the stats are still filled in).  Clamped corrections are counted
 * in unreached_faces and are not an error. */
vof_status vof_get_stats(vof_mesh *mesh, vof_stats *out);
vof_status vof_reset_stats(vof_mesh *mesh);

/* Block the host until the mesh's enqueued work is done; surfaces latched
 * device errors. */
vof_status vof_synchronize(vof_mesh *mesh);

/* Per-kernel timing.  While enabled, vof_advect brackets every kernel it
 * launches with HIP events on the context's stream.  vof_read_profile
 * synchronises, writes for kernel ids 0..n-1 the summed duration in ms and
 * the number of launches since the last read, and clears the totals.
 * vof_profile_kernel_name gives the name of a kernel id (NULL past the last). */
vof_status vof_profile_enable(vof_mesh *mesh, int32_t enable);
const char *vof_profile_kernel_name(int32_t id);
vof_status vof_read_profile(vof_mesh *mesh, double *ms, int64_t *launches, int32_t n);

/* ---- Batched form --------------------------------------------------------
 * Many independent meshes advanced by the same launches (the paper's
 * parallel runs split one mesh across processes, Section 4.2.2; here whole
 * meshes share each kernel launch).  A batch refers to meshes uploaded with
 * vof_mesh_upload, each with its alpha and velocity set; they stay owned by
 * the caller, keep their own state (alpha, statistics, face results: read
 * with the single-mesh calls) and must outlive the batch.  Every step of
 * vof_batch_advect is one replay of a captured graph whose kernels walk the
 * work of all meshes at once -- cell and face blocks, interface cells and
 * geometric face groups taken from one queue spanning every mesh -- and run
 * on each mesh's work the same code, in the same order, as vof_advect does:
 * every mesh's results are bitwise those of its own vof_advect with the same
 * schedule (the paper's serial-equals-parallel property, Section 4.2.2).  */
typedef struct vof_batch vof_batch;

/* Launch configuration of a batch step; it changes the speed of a step, never
 * its results.  Defaults: grid_flux 4096, grid_clip 4096, clip_claim 2,
 * grid_plane 2048, grid_cells 4096. */
typedef struct {
  int32_t grid_flux;   /* persistent blocks of the flux kernel (rounded up to 8) */
  int32_t grid_clip;   /* waves of the register clip                          */
  int32_t clip_claim;  /* face groups per claim of the register clip's queue  */
  int32_t grid_plane;  /* blocks (four waves) of the plane kernel             */
  int32_t grid_cells;  /* blocks of the cell, point and update kernels        */
} vof_batch_config;

/* meshes: n (1..VOF_MAX_BATCH) distinct meshes on the context's device.  The
 * batch runs on the context's stream.  Errors: VOF_EINVAL, VOF_ENOMEM,
 * VOF_EDEVICE. */
#define VOF_MAX_BATCH 256
vof_status vof_batch_create(vof_context *ctx, vof_mesh *const *meshes, int32_t n,
                            vof_batch **out);
vof_status vof_batch_destroy(vof_batch *batch);
/* Advance every mesh of the batch by n_steps steps; mesh i's step k has length
 * dt[i * n_steps + k] and velocity / flux scale scale[i * n_steps + k] (host
 * arrays, copied before return).  Each mesh must have alpha and velocity set
 * and wisp redistribution off.  Waits for earlier work on the meshes' own
 * streams, then returns with the steps enqueued on the batch's stream: call
 * vof_batch_synchronize before using a mesh through the single-mesh calls.
 * Errors: VOF_EINVAL, VOF_ENOMEM, VOF_EDEVICE. */
vof_status vof_batch_advect(vof_batch *batch, int32_t n_steps, const double *dt,
                            const double *scale);
/* Wait for the batch's steps; returns the first latched device error of any
 * mesh (VOF_ECAPACITY, VOF_ESTENCIL). */
vof_status vof_batch_synchronize(vof_batch *batch);
vof_status vof_batch_get_config(const vof_batch *batch, vof_batch_config *out);
vof_status vof_batch_set_config(vof_batch *batch, const vof_batch_config *config);

/* Autotuner of the batch's launch configuration.  Advances the batch by
 * n_steps steps exactly as vof_batch_advect would (same arguments, bitwise
 * the same results, since a configuration changes only the speed of a step),
 * launching them kernel by kernel with a different candidate configuration
 * per step and timing the kernels each parameter drives (HIP events); then
 * keeps, per parameter, the fastest candidate seen and sets it as the batch's
 * configuration (also written to *out when out is non-NULL).  With
 * cache_path non-NULL the configuration is cached in that JSON file under a
 * key made of the GPU target (e.g. gfx950) and the batch's size bucket (face
 * kinds present, nearest powers of two of its faces and meshes): a cached
 * entry is used without timing (the steps are still advanced, as one graph
 * each), and a tuned one is added or replaced.  Four steps time every
 * candidate once.  Errors: as vof_batch_advect; VOF_EINVAL if the cache
 * cannot be written. */
vof_status vof_autotune(vof_batch *batch, int32_t n_steps, const double *dt,
                        const double *scale, const char *cache_path, vof_batch_config *out);

/* ---- Served form ---------------------------------------------------------
 * A request loop over advection jobs of different meshes and lengths.  A job
 * is (mesh, alpha0, velocity, schedule of n_steps steps); the mesh is one
 * uploaded with vof_mesh_upload, whose addressing and geometry the job reads
 * (never writes) and which must outlive it -- any number of jobs may share a
 * mesh.  Each job gets its own state (alpha, planes, face results, scratch,
 * its copy of the inputs) in a device arena of a fixed size, the HBM budget
 * given at creation: jobs are admitted in arrival order while their state
 * fits the free budget (and at most VOF_MAX_BATCH are resident), stay
 * resident until their last step, and leave; the arena block is reused by the
 * next admitted job.  A worker thread runs ticks: one batched step (as
 * vof_batch_advect) of every resident job, so jobs that arrive while others
 * run join at the next tick and their steps share the launches (continuous
 * batching).  Every job's final alpha is bitwise that of vof_advect of the
 * same inputs on the mesh alone.  Meshes' parameters apply to their jobs;
 * wisps, narrow band and stencil check must be off.  All server work goes on
 * a stream of its own on the context's device. */
typedef struct vof_server vof_server;
typedef struct vof_job vof_job;

typedef struct {
  int64_t jobs_done;        /* jobs finished (their alpha copied to the host)  */
  int64_t jobs_waiting;     /* submitted, not yet admitted                     */
  int64_t face_fluxes;      /* sum over finished jobs of steps x faces with flux */
  int64_t ticks;            /* batched steps run                               */
  double latency_p50_s;     /* finish - submission, over finished jobs         */
  double latency_p99_s;
  double latency_max_s;
  double face_fluxes_per_s; /* face_fluxes / (last finish - first submission)  */
  int32_t max_resident;     /* most jobs resident at one tick                  */
  int64_t budget_bytes;     /* the arena                                       */
  int64_t peak_bytes;       /* most of it held at once                         */
} vof_server_stats;

/* Reserve hbm_budget_bytes of device memory (at least 1 MiB) and start the
 * worker.  Errors: VOF_EINVAL, VOF_ENOMEM, VOF_EDEVICE. */
vof_status vof_server_create(vof_context *ctx, int64_t hbm_budget_bytes, vof_server **out);
/* Queue a job: alpha0 (n_cells), U0c (3 n_cells, x y z interleaved), F0
 * (n_faces; step k uses scale[k] U0c, scale[k] F0 and length dt[k], k <
 * n_steps) -- host arrays, copied before return.  Returns at once with a
 * handle that must be passed to vof_server_wait.  Errors: VOF_EINVAL,
 * VOF_EBUSY (the job's state alone exceeds the budget, or 4096 jobs wait),
 * or the error that stopped the server. */
vof_status vof_server_submit(vof_server *server, vof_mesh *mesh, const double *alpha0,
                             const double *U0c, const double *F0, int32_t n_steps,
                             const double *dt, const double *scale, vof_job **job);
/* Block until the job has finished; copy its final alpha to alpha_out (host,
 * n_cells; may be NULL) and its latency (finish - submission, seconds) to
 * latency_s (may be NULL); release the job.  Returns VOF_ECAPACITY if one of
 * its clipped polytopes overflowed, or the error that stopped the server. */
vof_status vof_server_wait(vof_job *job, double *alpha_out, double *latency_s);
vof_status vof_server_get_stats(vof_server *server, vof_server_stats *out);
/* Finish every submitted job, stop the worker and release the arena.  Jobs
 * not waited for are released without their results. */
vof_status vof_server_destroy(vof_server *server);

/* Host self-test of the device geometry routines (compiled for the host as
 * well): volume of the tetrahedron (a, b, c, d) (12 doubles) intersected with
 * the half-spaces {n_k . x <= s_k} (4 doubles per plane).  Returns the volume
 * (a flat tetrahedron may give a round-off sized negative value), or NaN on
 * capacity overflow or a bad argument.  Needs no GPU. */
double vof_selftest_tet_clip(const double *tet, int32_t n_planes, const double *planes);

/* Host self-test of the register-only closed forms the clip kernels use for a
 * (tetrahedron, cell) pair bounded by at most four planes (Section 2.1: the
 * tetrahedron's kept part under each plane as one or three tetrahedra, the
 * last plane by the closed-form kept fraction).  Same arguments and result
 * as vof_selftest_tet_clip; NaN for n_planes > 4 or a bad argument.  For two
 * to four planes the result is the sum of the first plane's split terms as
 * the kernels add them when three lanes share a pair (four-plane pairs, and
 * three-plane pairs on hexahedral meshes), and NaN when it differs from the
 * one-lane recursion (the other pairs) by more than 1e-14 of the
 * tetrahedron's volume. */
double vof_selftest_tet_clip_closed(const double *tet, int32_t n_planes, const double *planes);

#ifdef __cplusplus
}
#endif
#endif /* VOF_H */
