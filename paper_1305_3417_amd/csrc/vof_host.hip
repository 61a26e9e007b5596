// vof_host.hip -- C ABI, mesh validation and addressing, orchestration.
//
// The host side validates the mesh, builds the integer addressing once
// (cell -> faces with owner/neighbour signs, point -> cells, face stencils)
// and owns every device buffer.  All geometry and every step of the flux
// path run in the kernels of vof_device.hip, enqueued on the context's
// stream; nothing here touches floating-point data of the method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vof_host_internal.h"

using namespace vof;

namespace vof {

namespace {
thread_local std::string g_err;
}  // namespace

vof_status fail(vof_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char *last_error() { return g_err.c_str(); }

vof_status flags_status(const uint32_t *d_flags) {
  uint32_t fl = 0;
  HIP_OR_FAIL(hipMemcpy(&fl, d_flags, sizeof fl, hipMemcpyDeviceToHost));
  if (fl & kFlagCapacity) return fail(VOF_ECAPACITY, "a clipped polytope exceeded its capacity");
  if (fl & kFlagLeak) return fail(VOF_ESTENCIL, "a flux polyhedron left its stencil");
  return VOF_OK;
}

}  // namespace vof


// Staging of the step schedule (dt, then scale) for vof_advect_noalloc, in a
// fixed array of the library rather than memory the mesh allocates.  In host
// code `scratch` names a host-side stand-in: its device address on each GPU
// is taken once with hipGetSymbolAddress (at context creation, with that
// device current) and only that address is handed to kernels and copies.
static __device__ __align__(256) double scratch[2 * VOF_NOALLOC_MAX_STEPS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {nullptr};

// the device address of `scratch` on the current device (once per device)
vof_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(VOF_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return VOF_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(VOF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }
  g_scratch[device] = (double *)ptr;
  return VOF_OK;
}

double *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace

namespace {

vof_status set_device(const vof_context *ctx) {
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  return VOF_OK;
}

// copy n elements to a host vector, from host or device memory
template <class T>
vof_status fetch(std::vector<T> &out, const T *src, int64_t n, int32_t memory) {
  out.resize((size_t)(n > 0 ? n : 0));
  if (n <= 0) return VOF_OK;
  if (!src) return fail(VOF_EINVAL, "null array");
  if (memory == VOF_HOST) {
    std::memcpy(out.data(), src, sizeof(T) * (size_t)n);
  } else {
    HIP_OR_FAIL(hipMemcpy(out.data(), src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost));
  }
  return VOF_OK;
}

template <class T>
vof_status to_device(T *dst, const T *src, int64_t n, int32_t memory, hipStream_t st) {
  if (n <= 0) return VOF_OK;
  if (!src) return fail(VOF_EINVAL, "null array");
  hipMemcpyKind kind = memory == VOF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  HIP_OR_FAIL(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)n, kind, st));
  if (memory == VOF_HOST) HIP_OR_FAIL(hipStreamSynchronize(st));
  return VOF_OK;
}

template <class T>
vof_status from_device(T *dst, const T *src, int64_t n, int32_t memory, hipStream_t st) {
  if (n <= 0) return VOF_OK;
  if (!dst) return fail(VOF_EINVAL, "null output array");
  hipMemcpyKind kind = memory == VOF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HIP_OR_FAIL(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)n, kind, st));
  HIP_OR_FAIL(hipStreamSynchronize(st));
  return VOF_OK;
}

vof_status check_memory(int32_t memory) {
  if (memory != VOF_HOST && memory != VOF_DEVICE)
    return fail(VOF_EINVAL, "memory must be VOF_HOST or VOF_DEVICE");
  return VOF_OK;
}

vof_status device_status(vof_mesh *m) { return vof::flags_status(m->ds.flags); }

vof_params default_params() {
  vof_params p;
  p.eps = 1e-12;
  p.correction_rtol = 1e-15;
  p.correction_max_iter = 50;
  p.position_tol = 1e-15;
  p.position_max_iter = 100;
  p.gradient_zero = 1e-8;
  p.check_stencil = 0;
  p.gradient = VOF_GRADIENT_NAG;
  p.narrow_band = 0;
  p.wisps = 0;
  return p;
}

void to_dparams(const vof_params &p, DParams &d) {
  d.eps = p.eps;
  d.corr_rtol = p.correction_rtol;
  d.corr_max_iter = p.correction_max_iter;
  d.pos_tol = p.position_tol;
  d.pos_max_iter = p.position_max_iter;
  d.grad_zero = p.gradient_zero;
  d.check_stencil = p.check_stencil;
  d.gradient = p.gradient;
  d.band = p.narrow_band;
  d.wisps = p.wisps;
}

vof_params from_dparams(const DParams &d) {
  vof_params p;
  p.eps = d.eps;
  p.correction_rtol = d.corr_rtol;
  p.correction_max_iter = d.corr_max_iter;
  p.position_tol = d.pos_tol;
  p.position_max_iter = d.pos_max_iter;
  p.gradient_zero = d.grad_zero;
  p.check_stencil = d.check_stencil;
  p.gradient = d.gradient;
  p.narrow_band = d.band;
  p.wisps = d.wisps;
  return p;
}

// The cells sharing a point with each cell (sorted, the cell itself left
// out): the stencil of the least-squares gradient, built once on the host
// from the addressing already on the device.
vof_status build_point_neighbours(vof_mesh *m) {
  const DMesh &dm = m->dm;
  const int64_t nc = dm.nc, nf = dm.nf, np = dm.np;
  std::vector<int32_t> cf_off(nc + 1), foff(nf + 1), pc_off(np + 1);
  std::vector<int32_t> cf, fpts, pc;
  HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
  HIP_OR_FAIL(hipMemcpy(cf_off.data(), dm.cf_off, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost));
  HIP_OR_FAIL(hipMemcpy(foff.data(), dm.foff, sizeof(int32_t) * (nf + 1), hipMemcpyDeviceToHost));
  HIP_OR_FAIL(hipMemcpy(pc_off.data(), dm.pc_off, sizeof(int32_t) * (np + 1), hipMemcpyDeviceToHost));
  cf.resize(cf_off[nc]);
  fpts.resize(foff[nf]);
  pc.resize(pc_off[np]);
  HIP_OR_FAIL(hipMemcpy(cf.data(), dm.cf, sizeof(int32_t) * cf.size(), hipMemcpyDeviceToHost));
  HIP_OR_FAIL(hipMemcpy(fpts.data(), dm.fpts, sizeof(int32_t) * fpts.size(), hipMemcpyDeviceToHost));
  HIP_OR_FAIL(hipMemcpy(pc.data(), dm.pc, sizeof(int32_t) * pc.size(), hipMemcpyDeviceToHost));
  auto gather = [&](int64_t c, std::vector<int32_t> &buf) {
    buf.clear();
    for (int32_t k = cf_off[c]; k < cf_off[c + 1]; ++k) {
      int32_t f = cf[k] >= 0 ? cf[k] : ~cf[k];
      for (int32_t i = foff[f]; i < foff[f + 1]; ++i)
        for (int32_t j = pc_off[fpts[i]]; j < pc_off[fpts[i] + 1]; ++j)
          if (pc[j] != c) buf.push_back(pc[j]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
  };
  std::vector<int32_t> cnt(nc);
#pragma omp parallel
  {
    std::vector<int32_t> buf;
#pragma omp for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
      gather(c, buf);
      cnt[c] = (int32_t)buf.size();
    }
  }
  std::vector<int32_t> off(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) {
    if (off[c] > INT32_MAX - cnt[c]) return fail(VOF_ENOMEM, "point-neighbour stencil too large");
    off[c + 1] = off[c] + cnt[c];
  }
  std::vector<int32_t> nb(off[nc]);
#pragma omp parallel
  {
    std::vector<int32_t> buf;
#pragma omp for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
      gather(c, buf);
      std::copy(buf.begin(), buf.end(), nb.begin() + off[c]);
    }
  }
  int32_t *d_off = nullptr, *d_nb = nullptr;
  vof_status rc;
  if ((rc = m->alloc(&d_off, nc + 1)) || (rc = m->alloc(&d_nb, (int64_t)nb.size()))) return rc;
  HIP_OR_FAIL(hipMemcpy(d_off, off.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice));
  if (!nb.empty())
    HIP_OR_FAIL(hipMemcpy(d_nb, nb.data(), sizeof(int32_t) * nb.size(), hipMemcpyHostToDevice));
  m->dm.cpn_off = d_off;
  m->dm.cpn = d_nb;
  return VOF_OK;
}

// Capture the launch sequence of one step on a private stream (the caller's
// stream may be the null stream, which cannot be captured), with the plane
// kernel on a side stream forked from and joined back into the capture.  The
// step contains kernels only: no memset or copy nodes.
vof_status build_step_graph(vof_mesh *m) {
  if (!m->cap_stream) HIP_OR_FAIL(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
  if (!m->fork.side) HIP_OR_FAIL(hipStreamCreateWithFlags(&m->fork.side, hipStreamNonBlocking));
  if (!m->fork.fork) HIP_OR_FAIL(hipEventCreateWithFlags(&m->fork.fork, hipEventDisableTiming));
  if (!m->fork.join) HIP_OR_FAIL(hipEventCreateWithFlags(&m->fork.join, hipEventDisableTiming));
  if (m->step_graph) {
    HIP_OR_FAIL(hipGraphExecDestroy(m->step_graph));
    m->step_graph = nullptr;
  }
  hipGraph_t g = nullptr;
  HIP_OR_FAIL(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
  launch_step(m->dm, m->ds, m->dp, m->cap_stream, nullptr, &m->fork);
  hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
  if (e != hipSuccess) return fail(VOF_EDEVICE, "step capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&m->step_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    m->step_graph = nullptr;
    return fail(VOF_EDEVICE, "step graph: %s", hipGetErrorString(e));
  }
  m->graph_ok = true;
  return VOF_OK;
}

}  // namespace

extern "C" {

const char *vof_last_error(void) { return vof::last_error(); }

const char *vof_version(void) { return "vofmi 0.1 (gfx950, fp64)"; }

vof_status vof_context_create(int32_t device, void *hip_stream, vof_context **out) {
  if (!out) return fail(VOF_EINVAL, "out is null");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(VOF_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= n) return fail(VOF_EINVAL, "device %d out of range", device);
  HIP_OR_FAIL(hipSetDevice(device));
  vof_status rc = scratch_init(device);
  if (rc) return rc;
  vof_context *c = new (std::nothrow) vof_context;
  if (!c) return fail(VOF_ENOMEM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return VOF_OK;
}

vof_status vof_context_destroy(vof_context *ctx) {
  delete ctx;
  return VOF_OK;
}

vof_status vof_mesh_upload(vof_context *ctx, const vof_mesh_desc *d, vof_mesh **out) {
  if (!ctx || !d || !out) return fail(VOF_EINVAL, "null argument");
  *out = nullptr;
  vof_status rc = check_memory(d->memory);
  if (rc) return rc;
  const int64_t np = d->n_points, nc = d->n_cells, nf = d->n_faces, ni = d->n_internal;
  if (np < 4 || nc < 1 || nf < 4 || ni < 0 || ni > nf)
    return fail(VOF_EBADMESH, "bad sizes (points %lld, cells %lld, faces %lld, internal %lld)",
                (long long)np, (long long)nc, (long long)nf, (long long)ni);
  if (np >= INT32_MAX || nc >= INT32_MAX || nf >= INT32_MAX)
    return fail(VOF_EBADMESH, "mesh too large for 32-bit indices");
  if ((rc = set_device(ctx))) return rc;

  std::vector<double> pts;
  std::vector<int64_t> foff64;
  std::vector<int32_t> fpts, own, nei;
  if ((rc = fetch(pts, d->points, 3 * np, d->memory))) return rc;
  if ((rc = fetch(foff64, d->face_offsets, nf + 1, d->memory))) return rc;
  if (foff64[0] != 0) return fail(VOF_EBADMESH, "face_offsets[0] must be 0");
  for (int64_t f = 0; f < nf; ++f) {
    int64_t n = foff64[f + 1] - foff64[f];
    if (n < 3 || n > VOF_MAX_FACE_POINTS)
      return fail(VOF_EBADMESH, "face %lld has %lld points (3..%d allowed)", (long long)f,
                  (long long)n, VOF_MAX_FACE_POINTS);
  }
  const int64_t nfp = foff64[nf];
  if (nfp >= INT32_MAX) return fail(VOF_EBADMESH, "too many face points");
  if ((rc = fetch(fpts, d->face_points, nfp, d->memory))) return rc;
  if ((rc = fetch(own, d->owner, nf, d->memory))) return rc;
  if ((rc = fetch(nei, d->neighbour, ni, d->memory))) return rc;
  for (int64_t k = 0; k < nfp; ++k)
    if (fpts[k] < 0 || fpts[k] >= np)
      return fail(VOF_EBADMESH, "face point index %d out of range", fpts[k]);
  for (int64_t f = 0; f < nf; ++f) {
    if (own[f] < 0 || own[f] >= nc) return fail(VOF_EBADMESH, "owner of face %lld out of range", (long long)f);
    if (f < ni && (nei[f] <= own[f] || nei[f] >= nc))
      return fail(VOF_EBADMESH, "neighbour of face %lld must exceed its owner and be < n_cells",
                  (long long)f);
  }
  for (int64_t k = 0; k < 3 * np; ++k)
    if (!std::isfinite(pts[k])) return fail(VOF_EBADMESH, "non-finite point coordinate");

  // cell -> faces (owner +f, neighbour ~f), faces in increasing order
  std::vector<int32_t> cf_off(nc + 1, 0), cf;
  for (int64_t f = 0; f < nf; ++f) {
    cf_off[own[f] + 1]++;
    if (f < ni) cf_off[nei[f] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) cf_off[c + 1] += cf_off[c];
  int32_t maxcf = 0;
  for (int64_t c = 0; c < nc; ++c) {
    int32_t k = cf_off[c + 1] - cf_off[c];
    if (k < 4) return fail(VOF_EBADMESH, "cell %lld has %d faces", (long long)c, k);
    maxcf = std::max(maxcf, k);
  }
  if (maxcf > kMaxCellPlanes)
    return fail(VOF_EBADMESH, "a cell has %d faces (at most %d supported)", maxcf, kMaxCellPlanes);
  cf.resize(cf_off[nc]);
  {
    std::vector<int32_t> fill(nc, 0);
    for (int64_t f = 0; f < nf; ++f) {
      cf[cf_off[own[f]] + fill[own[f]]++] = (int32_t)f;
      if (f < ni) cf[cf_off[nei[f]] + fill[nei[f]]++] = ~(int32_t)f;
    }
  }
  // face-fan tetrahedra of the largest cell (one per face point)
  int64_t maxslots = 0;
  for (int64_t c = 0; c < nc; ++c) {
    int64_t sl = 0;
    for (int32_t k = cf_off[c]; k < cf_off[c + 1]; ++k) {
      const int64_t f = cf[k] >= 0 ? cf[k] : ~cf[k];
      sl += foff64[f + 1] - foff64[f];
    }
    maxslots = std::max(maxslots, sl);
  }
  // point -> cells (sorted, unique)
  std::vector<int32_t> pc_off(np + 1, 0), pc;
  {
    std::vector<int64_t> cnt(np + 1, 0);
    for (int64_t f = 0; f < nf; ++f)
      for (int64_t k = foff64[f]; k < foff64[f + 1]; ++k) cnt[fpts[k] + 1] += (f < ni) ? 2 : 1;
    for (int64_t p = 0; p < np; ++p) cnt[p + 1] += cnt[p];
    std::vector<int32_t> tmp(cnt[np]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
      for (int64_t k = foff64[f]; k < foff64[f + 1]; ++k) {
        int32_t p = fpts[k];
        tmp[pos[p]++] = own[f];
        if (f < ni) tmp[pos[p]++] = nei[f];
      }
    std::vector<int32_t> ucount(np);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
      auto b = tmp.begin() + cnt[p], e = tmp.begin() + cnt[p + 1];
      std::sort(b, e);
      ucount[p] = (int32_t)(std::unique(b, e) - b);
    }
    for (int64_t p = 0; p < np; ++p) {
      if (ucount[p] == 0) return fail(VOF_EBADMESH, "point %lld is not used by any face", (long long)p);
      pc_off[p + 1] = pc_off[p] + ucount[p];
    }
    pc.resize(pc_off[np]);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p)
      std::copy(tmp.begin() + cnt[p], tmp.begin() + cnt[p] + ucount[p], pc.begin() + pc_off[p]);
  }
  // flux stencil of each face: the point-cells of its points (Section 2.3)
  std::vector<int32_t> st_off(nf + 1, 0), st;
  {
    std::vector<int32_t> scount(nf);
#pragma omp parallel
    {
      std::vector<int32_t> buf;
#pragma omp for schedule(static)
      for (int64_t f = 0; f < nf; ++f) {
        buf.clear();
        for (int64_t k = foff64[f]; k < foff64[f + 1]; ++k) {
          int32_t p = fpts[k];
          buf.insert(buf.end(), pc.begin() + pc_off[p], pc.begin() + pc_off[p + 1]);
        }
        std::sort(buf.begin(), buf.end());
        scount[f] = (int32_t)(std::unique(buf.begin(), buf.end()) - buf.begin());
      }
    }
    int64_t total = 0;
    for (int64_t f = 0; f < nf; ++f) {
      total += scount[f];
      if (total >= INT32_MAX) return fail(VOF_EBADMESH, "stencil too large for 32-bit offsets");
      st_off[f + 1] = (int32_t)total;
    }
    st.resize(total);
#pragma omp parallel
    {
      std::vector<int32_t> buf;
#pragma omp for schedule(static)
      for (int64_t f = 0; f < nf; ++f) {
        buf.clear();
        for (int64_t k = foff64[f]; k < foff64[f + 1]; ++k) {
          int32_t p = fpts[k];
          buf.insert(buf.end(), pc.begin() + pc_off[p], pc.begin() + pc_off[p + 1]);
        }
        std::sort(buf.begin(), buf.end());
        std::unique(buf.begin(), buf.end());
        std::copy(buf.begin(), buf.begin() + scount[f], st.begin() + st_off[f]);
      }
    }
  }
  std::vector<int32_t> foff(nf + 1);
  int32_t maxn = 0;
  for (int64_t f = 0; f <= nf; ++f) foff[f] = (int32_t)foff64[f];
  for (int64_t f = 0; f < nf; ++f) maxn = std::max(maxn, foff[f + 1] - foff[f]);

  vof_mesh *m = new (std::nothrow) vof_mesh;
  if (!m) return fail(VOF_ENOMEM, "host allocation failed");
  // the mesh keeps its own copy of the device and stream, so it stays usable
  // (and destroyable) after the context object is gone
  m->own_ctx = *ctx;
  m->ctx = &m->own_ctx;
  m->max_cell_faces = maxcf;
  m->st_entries = (int64_t)st.size();
  DMesh &dm = m->dm;
  DState &ds = m->ds;
  dm.np = np; dm.nc = nc; dm.nf = nf; dm.ni = ni;
  dm.maxn = maxn;
  dm.tpf = 5 * maxn;
  dm.wide = maxcf > 32 || maxslots > 64;
  hipStream_t s = ctx->stream;

  double4 *X, *S, *C, *XC, *cpl, *bblo, *bbhi;
  int32_t *d_foff, *d_fpts, *d_own, *d_nei, *d_cf_off, *d_cf, *d_pc_off, *d_pc, *d_st_off, *d_st;
  int32_t *d_fpad;
  // face points padded to a fixed width: one vector load per face
  const int32_t padw = maxn <= 4 ? 4 : 8;
  std::vector<int32_t> fpad((size_t)nf * padw, -1);
  for (int64_t f = 0; f < nf; ++f)
    for (int64_t k = foff[f]; k < foff[f + 1]; ++k) fpad[(size_t)f * padw + (k - foff[f])] = fpts[k];
  double *wpc, *V, *d_pts;
#define ALLOC(p, n) \
  do { if ((rc = m->alloc(&(p), (n)))) { delete m; return rc; } } while (0)
  ALLOC(X, np); ALLOC(d_pts, 3 * np); ALLOC(d_foff, nf + 1); ALLOC(d_fpts, nfp);
  ALLOC(d_fpad, nf * (int64_t)padw); ALLOC(ds.XU, 6 * np);
  ALLOC(d_own, nf); ALLOC(d_nei, ni); ALLOC(d_cf_off, nc + 1); ALLOC(d_cf, (int64_t)cf.size());
  ALLOC(d_pc_off, np + 1); ALLOC(d_pc, (int64_t)pc.size()); ALLOC(wpc, (int64_t)pc.size());
  ALLOC(d_st_off, nf + 1); ALLOC(d_st, (int64_t)st.size());
  ALLOC(S, nf); ALLOC(C, nf); ALLOC(V, nc); ALLOC(XC, nc); ALLOC(cpl, (int64_t)cf.size());
  uint8_t *npl, *isbox, *fan_w;
  ALLOC(npl, nc);
  ALLOC(isbox, nc);
  ALLOC(fan_w, nc);
  ALLOC(bblo, nc); ALLOC(bbhi, nc);
  ALLOC(ds.alpha, nc); ALLOC(ds.cls, nc); ALLOC(ds.plane, nc); ALLOC(ds.pmask, np);
  ALLOC(ds.alpha_p, np); ALLOC(ds.U, np); ALLOC(ds.F0, nf); ALLOC(ds.lam, nf);
  ALLOC(ds.vphase, nf); ALLOC(ds.vscale, nf); ALLOC(ds.coef, 3 * nf); ALLOC(ds.iters, nf); ALLOC(ds.kind, nf); ALLOC(ds.fstatus, nf);
  ALLOC(ds.icells, nc); ALLOC(ds.gfaces, nf); ALLOC(ds.tetvol, nf * (int64_t)dm.tpf);
  ALLOC(ds.defer, nf * (int64_t)dm.tpf);
  ALLOC(ds.stepno, 1); ALLOC(ds.work, kWNum); ALLOC(ds.cnt, kCntWords); ALLOC(ds.flags, 1); ALLOC(ds.ledger, 1);
  ALLOC(ds.part, (nc + 255) / 256 > 256 ? (nc + 255) / 256 : 256);
  ALLOC(m->stats_buf, 4);
#undef ALLOC
#define UP(dst, src, n)                                                                    \
  do { if ((rc = to_device(dst, src, n, VOF_HOST, s))) { delete m; return rc; } } while (0)
  UP(d_pts, pts.data(), 3 * np); UP(d_foff, foff.data(), nf + 1); UP(d_fpts, fpts.data(), nfp);
  UP(d_fpad, fpad.data(), nf * (int64_t)padw);
  UP(d_own, own.data(), nf); UP(d_nei, nei.data(), ni); UP(d_cf_off, cf_off.data(), nc + 1);
  UP(d_cf, cf.data(), (int64_t)cf.size()); UP(d_pc_off, pc_off.data(), np + 1);
  UP(d_pc, pc.data(), (int64_t)pc.size()); UP(d_st_off, st_off.data(), nf + 1);
  UP(d_st, st.data(), (int64_t)st.size());
#undef UP
  hipError_t e = hipMemsetAsync(ds.cnt, 0, sizeof(unsigned long long) * kCntWords, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.flags, 0, sizeof(uint32_t), s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.work, 0, sizeof(int32_t) * kWNum, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.ledger, 0, sizeof(double), s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.cls, 0, nc, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.plane, 0, sizeof(double4) * nc, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.alpha, 0, sizeof(double) * nc, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.U, 0, sizeof(double4) * np, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.XU, 0, sizeof(double) * 6 * np, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.F0, 0, sizeof(double) * nf, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.lam, 0, sizeof(double) * nf, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.vphase, 0, sizeof(double) * nf, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.iters, 0, nf, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.kind, 0, nf, s);
  if (e == hipSuccess) e = hipMemsetAsync(ds.fstatus, 0, nf, s);
  if (e != hipSuccess) { delete m; return fail(VOF_EDEVICE, "memset: %s", hipGetErrorString(e)); }
  dm.X = X; dm.foff = d_foff; dm.fpts = d_fpts; dm.own = d_own; dm.nei = d_nei;
  dm.fpad = d_fpad; dm.padw = padw;
  dm.cf_off = d_cf_off; dm.cf = d_cf; dm.pc_off = d_pc_off; dm.pc = d_pc; dm.wpc = wpc;
  dm.st_off = d_st_off; dm.st = d_st; dm.S = S; dm.C = C; dm.V = V; dm.XC = XC; dm.cpl = cpl; dm.npl = npl; dm.isbox = isbox; dm.fan_w = fan_w;
  dm.bblo = bblo; dm.bbhi = bbhi;
  launch_mesh_geometry(dm, X, d_pts, S, C, V, XC, wpc, cpl, npl, isbox, fan_w, bblo, bbhi,
                       ds.flags, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { delete m; return fail(VOF_EDEVICE, "mesh geometry: %s", hipGetErrorString(e)); }
  uint32_t fl = 0;
  e = hipMemcpy(&fl, ds.flags, sizeof fl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { delete m; return fail(VOF_EDEVICE, "%s", hipGetErrorString(e)); }
  if (fl & kFlagBadOrientation) {
    delete m;
    return fail(VOF_EBADMESH, "a face area vector does not point from owner to neighbour");
  }
  to_dparams(default_params(), m->dp);
  *out = m;
  return VOF_OK;
}

vof_status vof_mesh_destroy(vof_mesh *m) {
  if (!m) return VOF_OK;
  if (m->ctx) {
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream);
  }
  delete m;
  return VOF_OK;
}

vof_status vof_mesh_get_info(const vof_mesh *m, vof_mesh_info *out) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  out->n_points = m->dm.np;
  out->n_cells = m->dm.nc;
  out->n_faces = m->dm.nf;
  out->n_internal = m->dm.ni;
  out->stencil_entries = m->st_entries;
  out->max_face_points = m->dm.maxn;
  out->max_cell_faces = m->max_cell_faces;
  out->device_bytes = m->bytes;
  return VOF_OK;
}

vof_status vof_get_params(const vof_mesh *m, vof_params *out) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  *out = from_dparams(m->dp);
  return VOF_OK;
}

vof_status vof_set_params(vof_mesh *m, const vof_params *p) {
  if (!m || !p) return fail(VOF_EINVAL, "null argument");
  if (!(p->eps >= 0.0 && p->eps < 0.5)) return fail(VOF_EINVAL, "eps must be in [0, 0.5)");
  if (!(p->correction_rtol > 0.0) || p->correction_max_iter < 1 || p->correction_max_iter > 255)
    return fail(VOF_EINVAL, "bad correction tolerance or iteration limit (1..255)");
  if (!(p->position_tol > 0.0) || p->position_max_iter < 1)
    return fail(VOF_EINVAL, "bad positioning tolerance or iteration limit");
  if (!(p->gradient_zero >= 0.0)) return fail(VOF_EINVAL, "gradient_zero must be >= 0");
  if (p->gradient != VOF_GRADIENT_NAG && p->gradient != VOF_GRADIENT_LSQ)
    return fail(VOF_EINVAL, "gradient must be VOF_GRADIENT_NAG or VOF_GRADIENT_LSQ");
  if ((p->narrow_band != 0 && p->narrow_band != 1) || (p->wisps != 0 && p->wisps != 1))
    return fail(VOF_EINVAL, "narrow_band and wisps must be 0 or 1");
  if ((p->gradient == VOF_GRADIENT_LSQ || p->wisps) && !m->dm.cpn) {
    vof_status rc = set_device(m->ctx);
    if (rc || (rc = build_point_neighbours(m))) return rc;
  }
  if (p->check_stencil && !m->ds.tetdef) {
    // the stencil check keeps two more doubles per flux tet
    vof_status rc = set_device(m->ctx);
    if (rc) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
    if ((rc = m->alloc(&m->ds.tetdef, m->dm.nf * (int64_t)m->dm.tpf))) return rc;
    if ((rc = m->alloc(&m->ds.tetgross, m->dm.nf * (int64_t)m->dm.tpf))) return rc;
  }
  if (p->narrow_band && !m->ds.inexact) {
    vof_status rc = set_device(m->ctx);
    if (rc) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
    if ((rc = m->alloc(&m->ds.inexact, m->dm.nc)) || (rc = m->alloc(&m->ds.fbulk, m->dm.nf)))
      return rc;
  }
  if (p->wisps && !m->ds.wctr) {
    vof_status rc = set_device(m->ctx);
    if (rc) return rc;
    DState &d = m->ds;
    const int64_t nc = m->dm.nc;
    HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
    if ((rc = m->alloc(&d.wctr, 1)) || (rc = m->alloc(&d.wstamp, nc)) ||
        (rc = m->alloc(&d.rstamp, nc)) || (rc = m->alloc(&d.wlist, nc)) ||
        (rc = m->alloc(&d.rlist, nc)) || (rc = m->alloc(&d.wex, nc)) ||
        (rc = m->alloc(&d.wsum, nc)) || (rc = m->alloc(&d.rho, nc)))
      return rc;
    HIP_OR_FAIL(hipMemset(d.wctr, 0, sizeof(uint32_t)));
    HIP_OR_FAIL(hipMemset(d.wstamp, 0, sizeof(uint32_t) * nc));
    HIP_OR_FAIL(hipMemset(d.rstamp, 0, sizeof(uint32_t) * nc));
    HIP_OR_FAIL(hipDeviceSynchronize());
  }
  to_dparams(*p, m->dp);
  m->graph_ok = false;
  return VOF_OK;
}

vof_status vof_set_alpha(vof_mesh *m, const double *alpha, int32_t memory) {
  if (!m || !alpha) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  if ((rc = to_device(m->ds.alpha, alpha, m->dm.nc, memory, m->ctx->stream))) return rc;
  // the planes start from zero (the positioning's first estimate), so that a
  // run from a given alpha does not depend on what ran before
  HIP_OR_FAIL(hipMemsetAsync(m->ds.plane, 0, sizeof(double4) * (size_t)m->dm.nc, m->ctx->stream));
  m->have_alpha = true;
  return vof_reset_stats(m);
}

vof_status vof_map_alpha(vof_mesh *dst, vof_mesh *src, const int32_t *map_offsets,
                         const int32_t *map_cells, int32_t memory) {
  if (!dst || !src || !map_offsets || !map_cells) return fail(VOF_EINVAL, "null argument");
  if (dst == src) return fail(VOF_EINVAL, "source and destination meshes must differ");
  vof_status rc = check_memory(memory);
  if (rc) return rc;
  if (dst->ctx->device != src->ctx->device)
    return fail(VOF_EINVAL, "source and destination meshes are on different devices");
  if (!src->have_alpha) return fail(VOF_EINVAL, "source alpha not set");
  if ((rc = set_device(dst->ctx))) return rc;
  const int64_t nc = dst->dm.nc, onc = src->dm.nc;
  // temporary device buffers: the map (for host arrays) and a flag word
  struct Tmp {
    std::vector<void *> p;
    ~Tmp() { for (void *q : p) (void)hipFree(q); }
  } tmp;
  auto tmp_alloc = [&](size_t bytes, void **q) -> vof_status {
    hipError_t e = hipMalloc(q, bytes > 0 ? bytes : 1);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(VOF_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    tmp.p.push_back(*q);
    return VOF_OK;
  };
  const int32_t *off = map_offsets, *cells = map_cells;
  if (memory == VOF_HOST) {
    if (map_offsets[0] != 0) return fail(VOF_EINVAL, "map_offsets[0] must be 0");
    for (int64_t c = 0; c < nc; ++c)
      if (map_offsets[c + 1] <= map_offsets[c])
        return fail(VOF_EINVAL, "destination cell %lld has no source cell", (long long)c);
    const int64_t ne = map_offsets[nc];
    for (int64_t k = 0; k < ne; ++k)
      if (map_cells[k] < 0 || map_cells[k] >= onc)
        return fail(VOF_EINVAL, "map_cells[%lld] = %d out of range", (long long)k, map_cells[k]);
    void *a = nullptr, *b = nullptr;
    if ((rc = tmp_alloc(sizeof(int32_t) * (nc + 1), &a)) ||
        (rc = tmp_alloc(sizeof(int32_t) * ne, &b)))
      return rc;
    HIP_OR_FAIL(hipMemcpy(a, map_offsets, sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice));
    if (ne > 0) HIP_OR_FAIL(hipMemcpy(b, map_cells, sizeof(int32_t) * ne, hipMemcpyHostToDevice));
    off = (const int32_t *)a;
    cells = (const int32_t *)b;
  }
  void *fl = nullptr;
  if ((rc = tmp_alloc(sizeof(uint32_t), &fl))) return rc;
  HIP_OR_FAIL(hipMemset(fl, 0, sizeof(uint32_t)));
  // the old mesh's reconstruction of its current alpha, then the new alpha
  launch_reconstruct(src->dm, src->ds, src->dp, src->ctx->stream);
  HIP_OR_FAIL(hipGetLastError());
  HIP_OR_FAIL(hipStreamSynchronize(src->ctx->stream));
  hipStream_t st = dst->ctx->stream;
  launch_map_alpha(dst->dm, dst->ds.alpha, off, cells, src->dm, src->ds, (uint32_t *)fl, st);
  HIP_OR_FAIL(hipGetLastError());
  HIP_OR_FAIL(hipStreamSynchronize(st));
  uint32_t bad = 0;
  HIP_OR_FAIL(hipMemcpy(&bad, fl, sizeof bad, hipMemcpyDeviceToHost));
  if (bad) {
    dst->have_alpha = false;
    return fail(VOF_EINVAL, "a map entry is out of range or a destination cell has no entry");
  }
  HIP_OR_FAIL(hipMemsetAsync(dst->ds.plane, 0, sizeof(double4) * (size_t)nc, st));
  dst->have_alpha = true;
  return vof_reset_stats(dst);
}

vof_status vof_read_alpha(vof_mesh *m, double *out, int32_t memory) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  if ((rc = from_device(out, m->ds.alpha, m->dm.nc, memory, m->ctx->stream))) return rc;
  return device_status(m);
}

vof_status vof_set_velocity(vof_mesh *m, const double *U0c, const double *F0, int32_t memory) {
  if (!m || !U0c || !F0) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  hipStream_t s = m->ctx->stream;
  double *tmp = nullptr;
  HIP_OR_FAIL(hipMalloc(&tmp, sizeof(double) * 3 * (size_t)m->dm.nc));
  rc = to_device(tmp, U0c, 3 * m->dm.nc, memory, s);
  if (!rc) rc = to_device(m->ds.F0, F0, m->dm.nf, memory, s);
  if (!rc) {
    launch_point_velocity(m->dm, tmp, m->ds.U, m->ds.XU, m->ds.coef, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(VOF_EDEVICE, "point velocity: %s", hipGetErrorString(e));
  }
  (void)hipFree(tmp);
  if (!rc) m->have_velocity = true;
  return rc;
}

vof_status vof_reconstruct(vof_mesh *m) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  if (!m->have_alpha) return fail(VOF_EINVAL, "alpha not set");
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  launch_reconstruct(m->dm, m->ds, m->dp, m->ctx->stream);
  HIP_OR_FAIL(hipGetLastError());
  return VOF_OK;
}

vof_status vof_advect(vof_mesh *m, int32_t n_steps, const double *dt, const double *scale) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  if (n_steps < 0) return fail(VOF_EINVAL, "n_steps < 0");
  if (n_steps == 0) return VOF_OK;
  if (!dt || !scale) return fail(VOF_EINVAL, "null dt or scale");
  if (!m->have_alpha || !m->have_velocity) return fail(VOF_EINVAL, "alpha or velocity not set");
  for (int32_t i = 0; i < n_steps; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i]) || !std::isfinite(scale[i]))
      return fail(VOF_EINVAL, "dt must be positive and finite, scale finite (step %d)", i);
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  hipStream_t s = m->ctx->stream;
  if (n_steps > m->step_cap) {
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if ((rc = m->alloc(&m->ds.dt, n_steps))) return rc;
    if ((rc = m->alloc(&m->ds.sc, n_steps))) return rc;
    m->step_cap = n_steps;
    m->graph_ok = false;
  } else {
    HIP_OR_FAIL(hipStreamSynchronize(s));
  }
  HIP_OR_FAIL(hipMemcpy(m->ds.dt, dt, sizeof(double) * n_steps, hipMemcpyHostToDevice));
  HIP_OR_FAIL(hipMemcpy(m->ds.sc, scale, sizeof(double) * n_steps, hipMemcpyHostToDevice));
  const int32_t first = 0;
  HIP_OR_FAIL(hipMemcpy(m->ds.stepno, &first, sizeof first, hipMemcpyHostToDevice));
  if (m->profiling) {
    // room for every kernel of every step; pairs are folded into totals by
    // vof_read_profile
    int need = m->prof.n + n_steps * kKNum;
    if (need > m->prof.cap) {
      HIP_OR_FAIL(hipStreamSynchronize(s));
      Prof::Rec *nr = new (std::nothrow) Prof::Rec[need];
      if (!nr) return fail(VOF_ENOMEM, "host allocation failed");
      for (int i = 0; i < m->prof.cap; ++i) nr[i] = m->prof.recs[i];
      for (int i = m->prof.cap; i < need; ++i) {
        HIP_OR_FAIL(hipEventCreate(&nr[i].a));
        HIP_OR_FAIL(hipEventCreate(&nr[i].b));
      }
      delete[] m->prof.recs;
      m->prof.recs = nr;
      m->prof.cap = need;
    }
    m->prof.st = s;
  }
  if (m->profiling) {
    // kernel by kernel, each bracketed by timing events
    for (int32_t i = 0; i < n_steps; ++i) {
      launch_step(m->dm, m->ds, m->dp, s, &m->prof, nullptr);
      HIP_OR_FAIL(hipGetLastError());
    }
    return VOF_OK;
  }
  if (!m->graph_ok && (rc = build_step_graph(m))) return rc;
  for (int32_t i = 0; i < n_steps; ++i) HIP_OR_FAIL(hipGraphLaunch(m->step_graph, s));
  return VOF_OK;
}

vof_status vof_advect_noalloc(vof_mesh *m, int32_t n_steps, const double *dt,
                              const double *scale) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  if (n_steps < 0) return fail(VOF_EINVAL, "n_steps < 0");
  if (n_steps > VOF_NOALLOC_MAX_STEPS)
    return fail(VOF_EINVAL, "n_steps %d beyond the staging maximum of %d steps", n_steps,
                VOF_NOALLOC_MAX_STEPS);
  if (n_steps == 0) return VOF_OK;
  if (!dt || !scale) return fail(VOF_EINVAL, "null dt or scale");
  if (!m->have_alpha || !m->have_velocity) return fail(VOF_EINVAL, "alpha or velocity not set");
  for (int32_t i = 0; i < n_steps; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i]) || !std::isfinite(scale[i]))
      return fail(VOF_EINVAL, "dt must be positive and finite, scale finite (step %d)", i);
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  double *ptr = scratch_ptr(m->ctx->device);
  if (!ptr) return fail(VOF_EDEVICE, "staging buffer of device %d not set up", m->ctx->device);
  hipStream_t s = m->ctx->stream;
  // schedule and step counter staged in stream order behind earlier work of
  // this mesh; the host arrays may be reused once the call returns
  const int32_t first = 0;
  HIP_OR_FAIL(hipMemcpyAsync(ptr, dt, sizeof(double) * n_steps, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipMemcpyAsync(ptr + VOF_NOALLOC_MAX_STEPS, scale, sizeof(double) * n_steps,
                             hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipMemcpyAsync(m->ds.stepno, &first, sizeof first, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  DState ds = m->ds;
  ds.dt = ptr;
  ds.sc = ptr + VOF_NOALLOC_MAX_STEPS;
  // kernel by kernel on the mesh's stream (building a graph may allocate)
  for (int32_t i = 0; i < n_steps; ++i) {
    launch_step(m->dm, ds, m->dp, s, nullptr, nullptr);
    HIP_OR_FAIL(hipGetLastError());
  }
  return VOF_OK;
}

vof_status vof_read_face(vof_mesh *m, int32_t what, void *out, int32_t memory) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  hipStream_t s = m->ctx->stream;
  int64_t nf = m->dm.nf;
  switch (what) {
    case VOF_FACE_LAMBDA: rc = from_device((double *)out, m->ds.lam, nf, memory, s); break;
    case VOF_FACE_VPHASE: rc = from_device((double *)out, m->ds.vphase, nf, memory, s); break;
    case VOF_FACE_ITERS: rc = from_device((uint8_t *)out, m->ds.iters, nf, memory, s); break;
    case VOF_FACE_KIND: rc = from_device((uint8_t *)out, m->ds.kind, nf, memory, s); break;
    case VOF_FACE_STATUS: rc = from_device((uint8_t *)out, m->ds.fstatus, nf, memory, s); break;
    default: return fail(VOF_EINVAL, "unknown face field %d", what);
  }
  return rc;
}

vof_status vof_read_planes(vof_mesh *m, int8_t *cls, double *normal, double *sv, int32_t memory) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  hipStream_t s = m->ctx->stream;
  int64_t nc = m->dm.nc;
  if (cls && (rc = from_device(cls, m->ds.cls, nc, memory, s))) return rc;
  if (normal || sv) {
    std::vector<double4> pl(nc);
    if ((rc = from_device(pl.data(), m->ds.plane, nc, VOF_HOST, s))) return rc;
    std::vector<double> nn(normal ? 3 * nc : 0), ss(sv ? nc : 0);
    for (int64_t c = 0; c < nc; ++c) {
      if (normal) { nn[3 * c] = pl[c].x; nn[3 * c + 1] = pl[c].y; nn[3 * c + 2] = pl[c].z; }
      if (sv) ss[c] = pl[c].w;
    }
    if (normal && (rc = (memory == VOF_HOST)
                            ? (std::memcpy(normal, nn.data(), sizeof(double) * 3 * nc), VOF_OK)
                            : to_device(normal, nn.data(), 3 * nc, VOF_HOST, s)))
      return rc;
    if (sv && (rc = (memory == VOF_HOST) ? (std::memcpy(sv, ss.data(), sizeof(double) * nc), VOF_OK)
                                          : to_device(sv, ss.data(), nc, VOF_HOST, s)))
      return rc;
  }
  return VOF_OK;
}

vof_status vof_read_point_velocity(vof_mesh *m, double *out, int32_t memory) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  vof_status rc = check_memory(memory);
  if (rc || (rc = set_device(m->ctx))) return rc;
  int64_t np = m->dm.np;
  std::vector<double4> u(np);
  if ((rc = from_device(u.data(), m->ds.U, np, VOF_HOST, m->ctx->stream))) return rc;
  std::vector<double> o(3 * np);
  for (int64_t p = 0; p < np; ++p) { o[3 * p] = u[p].x; o[3 * p + 1] = u[p].y; o[3 * p + 2] = u[p].z; }
  if (memory == VOF_HOST) {
    std::memcpy(out, o.data(), sizeof(double) * 3 * np);
    return VOF_OK;
  }
  return to_device(out, o.data(), 3 * np, VOF_HOST, m->ctx->stream);
}

vof_status vof_synchronize(vof_mesh *m) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
  return device_status(m);
}

vof_status vof_get_stats(vof_mesh *m, vof_stats *out) {
  if (!m || !out) return fail(VOF_EINVAL, "null argument");
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  hipStream_t s = m->ctx->stream;
  launch_stats(m->dm, m->ds, m->stats_buf, s);
  HIP_OR_FAIL(hipGetLastError());
  std::vector<unsigned long long> slots(kCntWords);
  unsigned long long c[kCntNum] = {0};
  double st4[4], led = 0.0;
  if ((rc = from_device(slots.data(), m->ds.cnt, kCntWords, VOF_HOST, s))) return rc;
  for (int id = 0; id < kCntNum; ++id)
    for (int l = 0; l < kCntLanes; ++l) c[id] += slots[((int64_t)id * kCntLanes + l) * kCntStride];
  if ((rc = from_device(st4, m->stats_buf, 4, VOF_HOST, s))) return rc;
  if ((rc = from_device(&led, m->ds.ledger, 1, VOF_HOST, s))) return rc;
  out->steps = (int64_t)c[kCntSteps];
  out->face_fluxes = (int64_t)c[kCntFaceFluxes];
  out->geometric_faces = (int64_t)c[kCntGeometric];
  out->interface_cells = (int64_t)c[kCntInterface];
  out->fallback_cells = (int64_t)c[kCntFallback];
  out->unreached_faces = (int64_t)c[kCntUnreached];
  out->capacity_overflows = (int64_t)c[kCntCapacity];
  out->stencil_leaks = (int64_t)c[kCntLeaks];
  out->correction_iters = (int64_t)c[kCntIters];
  out->clip_pairs = (int64_t)c[kCntPairs];
  out->general_tets = (int64_t)c[kCntDeferred];
  out->ledger = led;
  out->mass = st4[0];
  out->alpha_min = st4[1];
  out->alpha_max = st4[2];
  out->wisps = (int64_t)c[kCntWisps];
  out->wisps_left = (int64_t)c[kCntWispsLeft];
  out->chunk_rescans = (int64_t)c[kCntRescans];
  return device_status(m);
}

vof_status vof_reset_stats(vof_mesh *m) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  hipStream_t s = m->ctx->stream;
  HIP_OR_FAIL(hipMemsetAsync(m->ds.cnt, 0, sizeof(unsigned long long) * kCntWords, s));
  HIP_OR_FAIL(hipMemsetAsync(m->ds.flags, 0, sizeof(uint32_t), s));
  HIP_OR_FAIL(hipMemsetAsync(m->ds.ledger, 0, sizeof(double), s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  return VOF_OK;
}

vof_status vof_profile_enable(vof_mesh *m, int32_t enable) {
  if (!m) return fail(VOF_EINVAL, "null argument");
  m->profiling = enable != 0;
  return VOF_OK;
}

const char *vof_profile_kernel_name(int32_t id) {
  static const char *names[kKNum] = {"reset",   "cell_class",   "point_prep", "plane",
                                     "flux",    "clip",         "clip_general", "face_sum",
                                     "update",  "ledger",       "wisps"};
  return (id >= 0 && id < kKNum) ? names[id] : nullptr;
}

vof_status vof_read_profile(vof_mesh *m, double *ms, int64_t *launches, int32_t n) {
  if (!m || !ms || !launches || n < 0) return fail(VOF_EINVAL, "null argument");
  vof_status rc = set_device(m->ctx);
  if (rc) return rc;
  HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
  for (int i = 0; i < m->prof.n; ++i) {
    float t = 0.0f;
    HIP_OR_FAIL(hipEventElapsedTime(&t, m->prof.recs[i].a, m->prof.recs[i].b));
    m->prof_ms[m->prof.recs[i].kid] += t;
    m->prof_count[m->prof.recs[i].kid] += 1;
  }
  m->prof.n = 0;
  for (int k = 0; k < n && k < kKNum; ++k) {
    ms[k] = m->prof_ms[k];
    launches[k] = m->prof_count[k];
  }
  for (int k = 0; k < kKNum; ++k) { m->prof_ms[k] = 0.0; m->prof_count[k] = 0; }
  return VOF_OK;
}

double vof_selftest_tet_clip(const double *tet, int32_t n_planes, const double *planes) {
  if (!tet || n_planes < 0 || (n_planes > 0 && !planes)) return NAN;
  return host_tet_clip(tet, n_planes, planes);
}

double vof_selftest_tet_clip_closed(const double *tet, int32_t n_planes, const double *planes) {
  if (!tet || n_planes < 0 || (n_planes > 0 && !planes)) return NAN;
  return host_tet_clip_closed(tet, n_planes, planes);
}

}  // extern "C"
