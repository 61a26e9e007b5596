// vof_systems.hip -- the batched and served forms of the flux path (host).
//
// Both run many meshes' steps through the same launches: a device table of
// the meshes' descriptors (addressing, state, parameters), rebuilt on the host
// when the set of meshes changes, and one captured graph per step that runs
// the batch kernels of vof_device.hip over the table.  Every mesh's results
// are those of its own plain run: the batch kernels execute the single-mesh
// kernels' code on each mesh's work, in the same order within each mesh.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "vof_host_internal.h"

using namespace vof;

namespace {

unsigned grid_blocks(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

BConf default_conf() {
  BConf c;
  c.grid_flux = 4096;
  c.grid_clip = 4096;
  c.clip_claim = 2;
  c.grid_plane = 2048;
  c.grid_cells = 4096;
  return c;
}

bool conf_valid(const vof_batch_config &c) {
  return c.grid_flux >= 8 && c.grid_flux <= 65536 && c.grid_clip >= 1 && c.grid_clip <= 65536 &&
         c.clip_claim >= 1 && c.clip_claim <= 64 && c.grid_plane >= 1 &&
         c.grid_plane <= 65536 && c.grid_cells >= 1 && c.grid_cells <= 65536;
}

BConf to_bconf(const vof_batch_config &c) {
  BConf b;
  b.grid_flux = c.grid_flux;
  b.grid_clip = c.grid_clip;
  b.clip_claim = c.clip_claim;
  b.grid_plane = c.grid_plane;
  b.grid_cells = c.grid_cells;
  return b;
}

vof_batch_config from_bconf(const BConf &b) {
  vof_batch_config c;
  c.grid_flux = b.grid_flux;
  c.grid_clip = b.grid_clip;
  c.clip_claim = b.clip_claim;
  c.grid_plane = b.grid_plane;
  c.grid_cells = b.grid_cells;
  return c;
}

// The device table of a set of meshes and the captured step over it.  The
// table lives in one device allocation; the host builds it in pinned memory
// and copies it in stream order, so steps already enqueued keep reading the
// old table until the copy runs.
struct BatchCore {
  int device = 0;
  hipStream_t stream = nullptr;  // the owner's stream
  void *dbase = nullptr;         // device table
  void *hbase = nullptr;         // pinned host image of the table
  size_t bytes = 0;
  hipEvent_t uploaded = nullptr;  // the last table copy has been read
  BTab tab{};
  BConf conf = default_conf();
  unsigned kinds = 0;
  int n = 0;
  // captured step per kinds mask (0..15: bits 0-2 the face kinds present, bit
  // 3 a mesh with whole-wave plane cells), valid for `conf`
  hipStream_t cap_stream = nullptr;
  Fork fork;
  hipGraphExec_t graph[16] = {nullptr};
  BConf graph_conf[16];

  // table layout (offsets into dbase / hbase)
  size_t o_hdr, o_inst, o_cls, o_pt, o_upd, o_klist, o_kflux, o_gpre, o_work;

  vof_status init(int dev, hipStream_t st) {
    device = dev;
    stream = st;
    size_t o = 0;
    auto take = [&](size_t n) {
      size_t at = o;
      o += (n + 255) / 256 * 256;
      return at;
    };
    o_hdr = take(sizeof(int32_t) * (1 + kFaceKinds));
    o_inst = take(sizeof(BInst) * kMaxBatch);
    o_cls = take(sizeof(int32_t) * (kMaxBatch + 1));
    o_pt = take(sizeof(int32_t) * (kMaxBatch + 1));
    o_upd = take(sizeof(int32_t) * (kMaxBatch + 1));
    o_klist = take(sizeof(int32_t) * kFaceKinds * kMaxBatch);
    o_kflux = take(sizeof(int32_t) * kFaceKinds * (kMaxBatch + 1));
    o_gpre = take(sizeof(int32_t) * kFaceKinds * (kMaxBatch + 1));
    o_work = take(sizeof(int32_t) * kBWNum);
    bytes = o;
    hipError_t e = hipMalloc(&dbase, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      dbase = nullptr;
      return fail(VOF_ENOMEM, "batch table: hipMalloc of %zu bytes failed", bytes);
    }
    HIP_OR_FAIL(hipHostMalloc(&hbase, bytes, hipHostMallocDefault));
    std::memset(hbase, 0, bytes);
    HIP_OR_FAIL(hipMemset(dbase, 0, bytes));
    HIP_OR_FAIL(hipEventCreateWithFlags(&uploaded, hipEventDisableTiming));
    char *d = (char *)dbase;
    tab.hdr = (const int32_t *)(d + o_hdr);
    tab.inst = (const BInst *)(d + o_inst);
    tab.cls_off = (const int32_t *)(d + o_cls);
    tab.pt_off = (const int32_t *)(d + o_pt);
    tab.upd_off = (const int32_t *)(d + o_upd);
    tab.klist = (const int32_t *)(d + o_klist);
    tab.kflux_off = (const int32_t *)(d + o_kflux);
    tab.gpre = (int32_t *)(d + o_gpre);
    tab.work = (int32_t *)(d + o_work);
    return VOF_OK;
  }

  // The meshes of the next steps (n <= kMaxBatch).  Enqueued on the stream.
  vof_status set(const BInst *entries, int count) {
    if (count < 0 || count > kMaxBatch) return fail(VOF_EINVAL, "at most %d meshes", kMaxBatch);
    // the pinned image may still be in flight from the previous set()
    HIP_OR_FAIL(hipEventSynchronize(uploaded));
    char *h = (char *)hbase;
    int32_t *hdr = (int32_t *)(h + o_hdr);
    BInst *inst = (BInst *)(h + o_inst);
    int32_t *cls = (int32_t *)(h + o_cls), *pt = (int32_t *)(h + o_pt), *upd = (int32_t *)(h + o_upd);
    int32_t *klist = (int32_t *)(h + o_klist), *kflux = (int32_t *)(h + o_kflux);
    n = count;
    kinds = 0;
    int kn[kFaceKinds] = {0, 0, 0};
    cls[0] = pt[0] = upd[0] = 0;
    for (int k = 0; k < kFaceKinds; ++k) kflux[k * (kMaxBatch + 1)] = 0;
    int64_t tc = 0, tp = 0, tu = 0, tf[kFaceKinds] = {0, 0, 0};
    for (int i = 0; i < count; ++i) {
      const BInst &b = entries[i];
      inst[i] = b;
      tc += grid_blocks(b.m.nc, 256 * 8);
      tp += grid_blocks(b.m.np, 256);
      tu += grid_blocks(b.m.nc, 256);
      const int k = face_kind(b.m.maxn);
      tf[k] += grid_blocks(b.m.nf, 256);
      if (tc >= INT32_MAX || tp >= INT32_MAX || tu >= INT32_MAX || tf[k] >= INT32_MAX)
        return fail(VOF_EINVAL, "batch too large");
      cls[i + 1] = (int32_t)tc;
      pt[i + 1] = (int32_t)tp;
      upd[i + 1] = (int32_t)tu;
      klist[k * kMaxBatch + kn[k]] = i;
      kflux[k * (kMaxBatch + 1) + kn[k] + 1] = (int32_t)tf[k];
      ++kn[k];
      kinds |= 1u << k;
      if (b.m.wide) kinds |= 8u;
    }
    hdr[0] = count;
    for (int k = 0; k < kFaceKinds; ++k) hdr[1 + k] = kn[k];
    // the claim counters are left as the last ledger cleared them (zero)
    HIP_OR_FAIL(hipMemcpyAsync(dbase, hbase, o_work, hipMemcpyHostToDevice, stream));
    HIP_OR_FAIL(hipEventRecord(uploaded, stream));
    return VOF_OK;
  }

  vof_status capture(unsigned mask) {
    if (!cap_stream) HIP_OR_FAIL(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    if (!fork.side) HIP_OR_FAIL(hipStreamCreateWithFlags(&fork.side, hipStreamNonBlocking));
    if (!fork.fork) HIP_OR_FAIL(hipEventCreateWithFlags(&fork.fork, hipEventDisableTiming));
    if (!fork.join) HIP_OR_FAIL(hipEventCreateWithFlags(&fork.join, hipEventDisableTiming));
    if (graph[mask]) {
      HIP_OR_FAIL(hipGraphExecDestroy(graph[mask]));
      graph[mask] = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_OR_FAIL(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    launch_batch_step(tab, conf, mask, kMaxBatch, cap_stream, &fork);
    hipError_t e = hipStreamEndCapture(cap_stream, &g);
    if (e != hipSuccess) return fail(VOF_EDEVICE, "batch step capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&graph[mask], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      graph[mask] = nullptr;
      return fail(VOF_EDEVICE, "batch step graph: %s", hipGetErrorString(e));
    }
    graph_conf[mask] = conf;
    return VOF_OK;
  }

  bool same_conf(const BConf &a, const BConf &b) const {
    return a.grid_flux == b.grid_flux && a.grid_clip == b.grid_clip &&
           a.clip_claim == b.clip_claim && a.grid_plane == b.grid_plane &&
           a.grid_cells == b.grid_cells;
  }

  // every mesh's step counter to 0 (before the first of a run of steps)
  vof_status begin() {
    launch_batch_begin(tab, n, stream);
    HIP_OR_FAIL(hipGetLastError());
    return VOF_OK;
  }

  // n_steps batch steps on the stream, each one replay of the captured step
  vof_status step(int32_t n_steps) {
    if (n == 0) return VOF_OK;
    vof_status rc;
    if (!graph[kinds] || !same_conf(graph_conf[kinds], conf))
      if ((rc = capture(kinds))) return rc;
    for (int32_t i = 0; i < n_steps; ++i) HIP_OR_FAIL(hipGraphLaunch(graph[kinds], stream));
    return VOF_OK;
  }

  // one step launched kernel by kernel (no graph), e.g. to time a configuration
  vof_status step_eager(const BConf &c, hipEvent_t *ev) {
    if (n == 0) return VOF_OK;
    launch_batch_step(tab, c, kinds, kMaxBatch, stream, nullptr, ev);
    HIP_OR_FAIL(hipGetLastError());
    return VOF_OK;
  }

  ~BatchCore() {
    for (auto &g : graph)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (fork.side) (void)hipStreamDestroy(fork.side);
    if (fork.fork) (void)hipEventDestroy(fork.fork);
    if (fork.join) (void)hipEventDestroy(fork.join);
    if (uploaded) (void)hipEventDestroy(uploaded);
    if (hbase) (void)hipHostFree(hbase);
    if (dbase) (void)hipFree(dbase);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
struct vof_batch {
  vof_context ctx{};
  std::vector<vof_mesh *> meshes;
  BatchCore core;
  double *sched = nullptr;  // dt of every mesh, then scale (n x cap each)
  int64_t sched_cap = 0;
  ~vof_batch() {
    if (sched) (void)hipFree(sched);
  }
};

extern "C" {

vof_status vof_batch_create(vof_context *ctx, vof_mesh *const *meshes, int32_t n,
                            vof_batch **out) {
  if (!ctx || !meshes || !out) return fail(VOF_EINVAL, "null argument");
  *out = nullptr;
  if (n < 1 || n > kMaxBatch) return fail(VOF_EINVAL, "a batch holds 1..%d meshes", kMaxBatch);
  for (int32_t i = 0; i < n; ++i) {
    const vof_mesh *m = meshes[i];
    if (!m) return fail(VOF_EINVAL, "mesh %d is null", i);
    if (m->ctx->device != ctx->device) return fail(VOF_EINVAL, "mesh %d is on another device", i);
    for (int32_t j = 0; j < i; ++j)
      if (meshes[j] == m) return fail(VOF_EINVAL, "mesh %d appears twice", i);
  }
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  vof_batch *b = new (std::nothrow) vof_batch;
  if (!b) return fail(VOF_ENOMEM, "host allocation failed");
  b->ctx = *ctx;
  b->meshes.assign(meshes, meshes + n);
  vof_status rc = b->core.init(ctx->device, ctx->stream);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return VOF_OK;
}

vof_status vof_batch_destroy(vof_batch *b) {
  if (!b) return VOF_OK;
  (void)hipSetDevice(b->ctx.device);
  (void)hipStreamSynchronize(b->ctx.stream);
  delete b;
  return VOF_OK;
}

vof_status vof_batch_get_config(const vof_batch *b, vof_batch_config *out) {
  if (!b || !out) return fail(VOF_EINVAL, "null argument");
  *out = from_bconf(b->core.conf);
  return VOF_OK;
}

vof_status vof_batch_set_config(vof_batch *b, const vof_batch_config *c) {
  if (!b || !c) return fail(VOF_EINVAL, "null argument");
  if (!conf_valid(*c)) return fail(VOF_EINVAL, "launch configuration out of range");
  b->core.conf = to_bconf(*c);
  return VOF_OK;
}

}  // extern "C"

namespace {

// Stage the schedule and the table for a run of n_steps batch steps.
vof_status batch_prepare(vof_batch *b, int32_t n_steps, const double *dt, const double *scale) {
  const int n = (int)b->meshes.size();
  if (n_steps < 0) return fail(VOF_EINVAL, "n_steps < 0");
  if (n_steps > 0 && (!dt || !scale)) return fail(VOF_EINVAL, "null dt or scale");
  for (int64_t k = 0; k < (int64_t)n * n_steps; ++k)
    if (!(dt[k] > 0.0) || !std::isfinite(dt[k]) || !std::isfinite(scale[k]))
      return fail(VOF_EINVAL, "dt must be positive and finite, scale finite (entry %lld)",
                  (long long)k);
  for (int i = 0; i < n; ++i) {
    vof_mesh *m = b->meshes[i];
    if (!m->have_alpha || !m->have_velocity)
      return fail(VOF_EINVAL, "mesh %d: alpha or velocity not set", i);
    if (m->dp.wisps) return fail(VOF_EINVAL, "mesh %d: wisp redistribution is not batched", i);
  }
  HIP_OR_FAIL(hipSetDevice(b->ctx.device));
  // the meshes' own earlier work (set_alpha and the like on their streams)
  for (vof_mesh *m : b->meshes) HIP_OR_FAIL(hipStreamSynchronize(m->ctx->stream));
  hipStream_t s = b->ctx.stream;
  HIP_OR_FAIL(hipStreamSynchronize(s));
  if (n_steps > b->sched_cap) {
    if (b->sched) HIP_OR_FAIL(hipFree(b->sched));
    b->sched = nullptr;
    b->sched_cap = 0;
    hipError_t e = hipMalloc(&b->sched, sizeof(double) * 2 * (size_t)n * n_steps);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b->sched = nullptr;
      return fail(VOF_ENOMEM, "batch schedule: hipMalloc failed");
    }
    b->sched_cap = n_steps;
  }
  const size_t per = sizeof(double) * (size_t)n * n_steps;
  if (n_steps > 0) {
    HIP_OR_FAIL(hipMemcpy(b->sched, dt, per, hipMemcpyHostToDevice));
    HIP_OR_FAIL(hipMemcpy(b->sched + (size_t)n * n_steps, scale, per, hipMemcpyHostToDevice));
  }
  std::vector<BInst> e(n);
  for (int i = 0; i < n; ++i) {
    vof_mesh *m = b->meshes[i];
    e[i].m = m->dm;
    e[i].s = m->ds;
    e[i].s.dt = b->sched + (size_t)i * n_steps;
    e[i].s.sc = b->sched + (size_t)n * n_steps + (size_t)i * n_steps;
    e[i].p = m->dp;
  }
  vof_status rc = b->core.set(e.data(), n);
  if (rc) return rc;
  return b->core.begin();
}

}  // namespace

extern "C" {

vof_status vof_batch_advect(vof_batch *b, int32_t n_steps, const double *dt, const double *scale) {
  if (!b) return fail(VOF_EINVAL, "null argument");
  if (n_steps == 0) return VOF_OK;
  vof_status rc = batch_prepare(b, n_steps, dt, scale);
  if (rc) return rc;
  return b->core.step(n_steps);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

// Candidate values of each tuned parameter, tried coordinate by coordinate.
// Each parameter drives its own kernels, so one step can time a candidate of
// every parameter at once: step k of a round uses candidate k of each list.
const int kCandFlux[] = {1024, 2048, 4096, 8192};
const int kCandClip[] = {2048, 4096, 8192, 16384};
const int kCandClaim[] = {1, 2, 4, 2};
const int kCandPlane[] = {1024, 2048, 4096, 2048};
const int kCandCells[] = {1024, 2048, 4096, 8192};
constexpr int kCands = 4;

std::string gpu_target(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// size bucket: face kinds present, and powers of two of faces and meshes
std::string bucket_key(const vof_batch *b, const std::string &target) {
  int64_t faces = 0;
  unsigned kinds = 0;
  for (const vof_mesh *m : b->meshes) {
    faces += m->dm.nf;
    kinds |= 1u << face_kind(m->dm.maxn);
  }
  auto lg = [](int64_t v) { return (int)std::lround(std::log2((double)std::max<int64_t>(v, 1))); };
  char buf[160];
  snprintf(buf, sizeof buf, "%s/kinds%u/faces2^%d/meshes2^%d", target.c_str(), kinds, lg(faces),
           lg((int64_t)b->meshes.size()));
  return buf;
}

// The cache: a JSON object, one entry per line, keyed by bucket.
struct CacheEntry {
  std::string key;
  vof_batch_config c;
};

std::vector<CacheEntry> cache_read(const char *path) {
  std::vector<CacheEntry> out;
  FILE *f = fopen(path, "r");
  if (!f) return out;
  char line[512], key[256];
  while (fgets(line, sizeof line, f)) {
    vof_batch_config c;
    if (sscanf(line,
               " \"%255[^\"]\": {\"grid_flux\": %d, \"grid_clip\": %d, \"clip_claim\": %d, "
               "\"grid_plane\": %d, \"grid_cells\": %d}",
               key, &c.grid_flux, &c.grid_clip, &c.clip_claim, &c.grid_plane,
               &c.grid_cells) == 6 &&
        conf_valid(c))
      out.push_back({key, c});
  }
  fclose(f);
  return out;
}

vof_status cache_write(const char *path, const std::vector<CacheEntry> &entries) {
  std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return fail(VOF_EINVAL, "cannot write the autotuning cache %s", tmp.c_str());
  fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i) {
    const vof_batch_config &c = entries[i].c;
    fprintf(f,
            "\"%s\": {\"grid_flux\": %d, \"grid_clip\": %d, \"clip_claim\": %d, "
            "\"grid_plane\": %d, \"grid_cells\": %d}%s\n",
            entries[i].key.c_str(), c.grid_flux, c.grid_clip, c.clip_claim, c.grid_plane,
            c.grid_cells, i + 1 < entries.size() ? "," : "");
  }
  fprintf(f, "}\n");
  if (fclose(f) != 0 || rename(tmp.c_str(), path) != 0)
    return fail(VOF_EINVAL, "cannot write the autotuning cache %s", path);
  return VOF_OK;
}

}  // namespace

extern "C" {

vof_status vof_autotune(vof_batch *b, int32_t n_steps, const double *dt, const double *scale,
                        const char *cache_path, vof_batch_config *out) {
  if (!b) return fail(VOF_EINVAL, "null argument");
  if (n_steps < 1) return fail(VOF_EINVAL, "the autotuner needs at least one step");
  vof_status rc = batch_prepare(b, n_steps, dt, scale);
  if (rc) return rc;
  const std::string key = bucket_key(b, gpu_target(b->ctx.device));
  std::vector<CacheEntry> cache;
  if (cache_path) {
    cache = cache_read(cache_path);
    for (const CacheEntry &e : cache)
      if (e.key == key) {
        b->core.conf = to_bconf(e.c);
        if (out) *out = e.c;
        return b->core.step(n_steps);
      }
  }
  hipEvent_t ev[8];
  for (auto &e : ev) HIP_OR_FAIL(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *ev;
    ~EvGuard() {
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
    }
  } guard{ev};
  // best time per candidate of each parameter (ms)
  float best[5][kCands];
  for (auto &r : best)
    for (float &x : r) x = 1e30f;
  hipStream_t s = b->ctx.stream;
  for (int32_t k = 0; k < n_steps; ++k) {
    const int j = k % kCands;
    BConf c;
    c.grid_flux = kCandFlux[j];
    c.grid_clip = kCandClip[j];
    c.clip_claim = kCandClaim[j];
    c.grid_plane = kCandPlane[j];
    c.grid_cells = kCandCells[j];
    rc = b->core.step_eager(c, ev);
    if (rc) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(s));
    float t[7];
    for (int i = 0; i < 7; ++i) HIP_OR_FAIL(hipEventElapsedTime(&t[i], ev[i], ev[i + 1]));
    const float cells = t[0] + t[5], plane = t[1], flux = t[2], clip = t[3];
    best[0][j] = std::min(best[0][j], flux);
    best[1][j] = std::min(best[1][j], clip);
    best[2][j] = std::min(best[2][j], clip);
    best[3][j] = std::min(best[3][j], plane);
    best[4][j] = std::min(best[4][j], cells);
  }
  auto pick = [&](int p, const int *vals, int dflt) {
    int arg = -1;
    for (int j = 0; j < kCands; ++j)
      if (best[p][j] < 1e29f && (arg < 0 || best[p][j] < best[p][arg])) arg = j;
    return arg < 0 ? dflt : vals[arg];
  };
  BConf c = default_conf();
  c.grid_flux = pick(0, kCandFlux, c.grid_flux);
  // the clip's grid and claim size were varied together; keep the pair
  int jc = -1;
  for (int j = 0; j < kCands; ++j)
    if (best[1][j] < 1e29f && (jc < 0 || best[1][j] < best[1][jc])) jc = j;
  if (jc >= 0) {
    c.grid_clip = kCandClip[jc];
    c.clip_claim = kCandClaim[jc];
  }
  c.grid_plane = pick(3, kCandPlane, c.grid_plane);
  c.grid_cells = pick(4, kCandCells, c.grid_cells);
  b->core.conf = c;
  const vof_batch_config vc = from_bconf(c);
  if (out) *out = vc;
  if (cache_path) {
    bool found = false;
    for (CacheEntry &e : cache)
      if (e.key == key) {
        e.c = vc;
        found = true;
      }
    if (!found) cache.push_back({key, vc});
    if ((rc = cache_write(cache_path, cache))) return rc;
  }
  return VOF_OK;
}

vof_status vof_batch_synchronize(vof_batch *b) {
  if (!b) return fail(VOF_EINVAL, "null argument");
  HIP_OR_FAIL(hipSetDevice(b->ctx.device));
  HIP_OR_FAIL(hipStreamSynchronize(b->ctx.stream));
  for (vof_mesh *m : b->meshes) {
    vof_status rc = flags_status(m->ds.flags);
    if (rc) return rc;
  }
  return VOF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// served form
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// The per-job state of a mesh (everything a step writes, and the job's own
// inputs) laid out in one block of the server's arena.
struct StateLayout {
  size_t alpha, cls, plane, pmask, alpha_p, U, XU, F0, coef, lam, vphase, vscale, iters, kind, fstatus,
      icells, gfaces, tetvol, defer, work, cnt, flags, ledger, part, stepno, dt, sc, bytes;
};

StateLayout state_layout(const DMesh &m, int64_t steps) {
  StateLayout L;
  size_t o = 0;
  auto take = [&](size_t n) {
    size_t at = o;
    o += align_up(n > 0 ? n : 1);
    return at;
  };
  const size_t nc = (size_t)m.nc, np = (size_t)m.np, nf = (size_t)m.nf, tpf = (size_t)m.tpf;
  L.alpha = take(8 * nc);
  L.cls = take(nc);
  L.plane = take(32 * nc);
  L.pmask = take(np);
  L.alpha_p = take(8 * np);
  L.U = take(32 * np);
  L.XU = take(48 * np);
  L.F0 = take(8 * nf);
  L.coef = take(24 * nf);
  L.lam = take(8 * nf);
  L.vphase = take(8 * nf);
  L.vscale = take(8 * nf);
  L.iters = take(nf);
  L.kind = take(nf);
  L.fstatus = take(nf);
  L.icells = take(4 * nc);
  L.gfaces = take(4 * nf);
  L.tetvol = take(8 * nf * tpf);
  L.defer = take(4 * nf * tpf);
  L.work = take(4 * kWNum);
  L.cnt = take(8 * (size_t)kCntWords);
  L.flags = take(4);
  L.ledger = take(8);
  const size_t nparts = std::max<size_t>((nc + 255) / 256, 256);
  L.part = take(8 * nparts);
  L.stepno = take(4);
  L.dt = take(8 * (size_t)steps);
  L.sc = take(8 * (size_t)steps);
  L.bytes = o;
  return L;
}

DState state_at(const StateLayout &L, char *b) {
  DState s{};
  s.alpha = (double *)(b + L.alpha);
  s.cls = (int8_t *)(b + L.cls);
  s.plane = (double4 *)(b + L.plane);
  s.pmask = (uint8_t *)(b + L.pmask);
  s.alpha_p = (double *)(b + L.alpha_p);
  s.U = (double4 *)(b + L.U);
  s.XU = (double *)(b + L.XU);
  s.F0 = (double *)(b + L.F0);
  s.coef = (double *)(b + L.coef);
  s.lam = (double *)(b + L.lam);
  s.vphase = (double *)(b + L.vphase);
  s.vscale = (double *)(b + L.vscale);
  s.iters = (uint8_t *)(b + L.iters);
  s.kind = (uint8_t *)(b + L.kind);
  s.fstatus = (uint8_t *)(b + L.fstatus);
  s.icells = (int32_t *)(b + L.icells);
  s.gfaces = (int32_t *)(b + L.gfaces);
  s.tetvol = (double *)(b + L.tetvol);
  s.defer = (int32_t *)(b + L.defer);
  s.work = (int32_t *)(b + L.work);
  s.cnt = (unsigned long long *)(b + L.cnt);
  s.flags = (uint32_t *)(b + L.flags);
  s.ledger = (double *)(b + L.ledger);
  s.part = (double *)(b + L.part);
  s.stepno = (int32_t *)(b + L.stepno);
  s.dt = (double *)(b + L.dt);
  s.sc = (double *)(b + L.sc);
  return s;
}

// First-fit allocator over the server's budget (offsets, kAlign multiples).
struct Arena {
  size_t size = 0, used = 0, peak = 0;
  std::vector<std::pair<size_t, size_t>> free_;  // (offset, length), sorted, coalesced
  void init(size_t n) {
    size = n / kAlign * kAlign;
    free_.assign(1, {0, size});
  }
  bool alloc(size_t n, size_t &off) {
    n = align_up(n);
    for (size_t i = 0; i < free_.size(); ++i)
      if (free_[i].second >= n) {
        off = free_[i].first;
        free_[i].first += n;
        free_[i].second -= n;
        if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    used -= n;
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
    it = free_.insert(it, {off, n});
    size_t i = (size_t)(it - free_.begin());
    if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
      free_[i].second += free_[i + 1].second;
      free_.erase(free_.begin() + (long)i + 1);
    }
    if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
      free_[i - 1].second += free_[i].second;
      free_.erase(free_.begin() + (long)i);
    }
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

enum JobState { kPending = 0, kResident, kDraining, kDone };

}  // namespace

struct vof_job {
  vof_server *srv = nullptr;
  vof_mesh *mesh = nullptr;
  std::vector<double> alpha0, U0c, F0, dt, sc;
  int32_t steps = 0, done_steps = 0;
  int64_t nflux = 0;
  StateLayout L{};
  size_t off = 0;
  DState ds{};
  double *h_out = nullptr;  // pinned: alpha, then the flags word
  hipEvent_t ev = nullptr;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  JobState state = kPending;
  vof_status status = VOF_OK;
};

struct vof_server {
  vof_context ctx{};
  hipStream_t stream = nullptr;
  char *arena_base = nullptr;
  Arena arena;
  BatchCore core;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<vof_job *> pending;
  std::vector<vof_job *> resident, draining;
  bool stop = false;
  vof_status error = VOF_OK;
  std::string error_msg;
  // statistics (under mu)
  std::vector<double> latencies;
  int64_t face_fluxes = 0, jobs_done = 0, ticks = 0;
  int32_t max_resident = 0;
  double t_first_arrival = -1, t_last_done = 0;
  hipEvent_t tick_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int tick_slot = 0;
};

namespace {

// Stage a job's inputs into its block of the arena (in stream order).
vof_status job_admit(vof_server *S, vof_job *j) {
  hipStream_t s = S->stream;
  j->ds = state_at(j->L, S->arena_base + j->off);
  const DMesh &m = j->mesh->dm;
  DState &d = j->ds;
  HIP_OR_FAIL(hipMemsetAsync(d.work, 0, 4 * kWNum, s));
  HIP_OR_FAIL(hipMemsetAsync(d.cnt, 0, 8 * (size_t)kCntWords, s));
  HIP_OR_FAIL(hipMemsetAsync(d.flags, 0, 4, s));
  HIP_OR_FAIL(hipMemsetAsync(d.ledger, 0, 8, s));
  HIP_OR_FAIL(hipMemsetAsync(d.stepno, 0, 4, s));
  HIP_OR_FAIL(hipMemsetAsync(d.cls, 0, (size_t)m.nc, s));
  HIP_OR_FAIL(hipMemsetAsync(d.plane, 0, 32 * (size_t)m.nc, s));
  HIP_OR_FAIL(hipMemsetAsync(d.lam, 0, 8 * (size_t)m.nf, s));
  HIP_OR_FAIL(hipMemsetAsync(d.vphase, 0, 8 * (size_t)m.nf, s));
  HIP_OR_FAIL(hipMemcpyAsync(d.alpha, j->alpha0.data(), 8 * (size_t)m.nc, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipMemcpyAsync(d.F0, j->F0.data(), 8 * (size_t)m.nf, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipMemcpyAsync(d.dt, j->dt.data(), 8 * (size_t)j->steps, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipMemcpyAsync(d.sc, j->sc.data(), 8 * (size_t)j->steps, hipMemcpyHostToDevice, s));
  // the cell velocities are staged in the (not yet used) flux-tet slots
  double *U0c = d.tetvol;
  HIP_OR_FAIL(hipMemcpyAsync(U0c, j->U0c.data(), 24 * (size_t)m.nc, hipMemcpyHostToDevice, s));
  launch_point_velocity(m, U0c, d.U, d.XU, d.coef, s);
  HIP_OR_FAIL(hipGetLastError());
  HIP_OR_FAIL(hipHostMalloc((void **)&j->h_out, 8 * (size_t)m.nc + 8, hipHostMallocDefault));
  HIP_OR_FAIL(hipEventCreateWithFlags(&j->ev, hipEventDisableTiming));
  // the host inputs were copied from pageable memory before the calls returned
  std::vector<double>().swap(j->alpha0);
  std::vector<double>().swap(j->U0c);
  std::vector<double>().swap(j->F0);
  return VOF_OK;
}

// Enqueue the copy of a finished job's alpha and flags to its pinned buffer.
vof_status job_drain(vof_server *S, vof_job *j) {
  const size_t nc = (size_t)j->mesh->dm.nc;
  HIP_OR_FAIL(hipMemcpyAsync(j->h_out, j->ds.alpha, 8 * nc, hipMemcpyDeviceToHost, S->stream));
  HIP_OR_FAIL(hipMemcpyAsync(j->h_out + nc, j->ds.flags, 4, hipMemcpyDeviceToHost, S->stream));
  HIP_OR_FAIL(hipEventRecord(j->ev, S->stream));
  return VOF_OK;
}

vof_status server_loop_once(vof_server *S, bool &idle) {
  idle = false;
  // finished copies: the jobs are done
  {
    std::vector<vof_job *> still;
    for (vof_job *j : S->draining) {
      hipError_t q = hipEventQuery(j->ev);
      if (q == hipErrorNotReady) {
        still.push_back(j);
        continue;
      }
      if (q != hipSuccess) return fail(VOF_EDEVICE, "server: %s", hipGetErrorString(q));
      uint32_t fl = 0;
      std::memcpy(&fl, j->h_out + j->mesh->dm.nc, 4);
      std::lock_guard<std::mutex> lock(S->mu);
      j->t_done = now_s();
      j->status = (fl & kFlagCapacity) ? VOF_ECAPACITY : VOF_OK;
      j->state = kDone;
      S->latencies.push_back(j->t_done - j->t_arrive);
      S->face_fluxes += j->nflux * j->steps;
      ++S->jobs_done;
      S->t_last_done = j->t_done;
      S->cv_done.notify_all();
    }
    S->draining.swap(still);
  }
  // admission, first come first served, while the budget and the table allow
  bool changed = false;
  for (;;) {
    vof_job *j = nullptr;
    {
      std::lock_guard<std::mutex> lock(S->mu);
      if (S->pending.empty() || (int)S->resident.size() >= kMaxBatch) break;
      j = S->pending.front();
      size_t off = 0;
      if (!S->arena.alloc(j->L.bytes, off)) break;
      j->off = off;
      S->pending.pop_front();
      j->state = kResident;
      j->t_admit = now_s();
    }
    vof_status rc = job_admit(S, j);
    if (rc) return rc;
    S->resident.push_back(j);
    changed = true;
  }
  if (S->resident.empty()) {
    idle = true;
    return VOF_OK;
  }
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->max_resident = std::max(S->max_resident, (int32_t)S->resident.size());
  }
  if (changed || S->core.n != (int)S->resident.size()) {
    std::vector<BInst> e(S->resident.size());
    for (size_t i = 0; i < S->resident.size(); ++i) {
      e[i].m = S->resident[i]->mesh->dm;
      e[i].s = S->resident[i]->ds;
      e[i].p = S->resident[i]->mesh->dp;
    }
    vof_status rc = S->core.set(e.data(), (int)e.size());
    if (rc) return rc;
  }
  // one batched step of every resident job; at most four ticks in flight
  hipEvent_t &ev = S->tick_ev[S->tick_slot];
  if (S->ticks >= 4) HIP_OR_FAIL(hipEventSynchronize(ev));
  vof_status rc = S->core.step(1);
  if (rc) return rc;
  HIP_OR_FAIL(hipEventRecord(ev, S->stream));
  S->tick_slot = (S->tick_slot + 1) % 4;
  ++S->ticks;
  std::vector<vof_job *> still;
  for (vof_job *j : S->resident) {
    if (++j->done_steps < j->steps) {
      still.push_back(j);
      continue;
    }
    if ((rc = job_drain(S, j))) return rc;
    {
      std::lock_guard<std::mutex> lock(S->mu);
      // later uploads into this block are ordered after the copy on the stream
      S->arena.release(j->off, j->L.bytes);
      j->state = kDraining;
    }
    S->draining.push_back(j);
  }
  S->resident.swap(still);
  return VOF_OK;
}

void server_worker(vof_server *S) {
  if (hipSetDevice(S->ctx.device) != hipSuccess) {
    std::lock_guard<std::mutex> lock(S->mu);
    S->error = VOF_EDEVICE;
    S->error_msg = "server: hipSetDevice failed";
    S->cv_done.notify_all();
    return;
  }
  for (;;) {
    bool idle = false;
    vof_status rc = server_loop_once(S, idle);
    if (rc) {
      std::lock_guard<std::mutex> lock(S->mu);
      S->error = rc;
      S->error_msg = last_error();
      S->cv_done.notify_all();
      return;
    }
    if (idle) {
      if (!S->draining.empty()) {
        // nothing to step: wait for the oldest copy
        (void)hipEventSynchronize(S->draining.front()->ev);
        continue;
      }
      std::unique_lock<std::mutex> lock(S->mu);
      if (S->stop && S->pending.empty()) return;
      S->cv_work.wait(lock, [&] { return S->stop || !S->pending.empty(); });
      if (S->stop && S->pending.empty()) return;
    }
  }
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

vof_status vof_server_create(vof_context *ctx, int64_t hbm_budget_bytes, vof_server **out) {
  if (!ctx || !out) return fail(VOF_EINVAL, "null argument");
  *out = nullptr;
  if (hbm_budget_bytes < (int64_t)(1 << 20)) return fail(VOF_EINVAL, "budget below 1 MiB");
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  vof_server *S = new (std::nothrow) vof_server;
  if (!S) return fail(VOF_ENOMEM, "host allocation failed");
  S->ctx = *ctx;
  auto bail = [&](vof_status rc) {
    if (S->stream) (void)hipStreamDestroy(S->stream);
    if (S->arena_base) (void)hipFree(S->arena_base);
    for (auto &e : S->tick_ev)
      if (e) (void)hipEventDestroy(e);
    delete S;
    return rc;
  };
  hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(fail(VOF_EDEVICE, "server stream: %s", hipGetErrorString(e)));
  e = hipMalloc((void **)&S->arena_base, (size_t)hbm_budget_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    S->arena_base = nullptr;
    return bail(fail(VOF_ENOMEM, "server budget: hipMalloc of %lld bytes failed",
                     (long long)hbm_budget_bytes));
  }
  S->arena.init((size_t)hbm_budget_bytes);
  for (auto &ev : S->tick_ev) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return bail(fail(VOF_EDEVICE, "server events: %s", hipGetErrorString(e)));
  }
  vof_status rc = S->core.init(ctx->device, S->stream);
  if (rc) return bail(rc);
  S->worker = std::thread(server_worker, S);
  *out = S;
  return VOF_OK;
}

vof_status vof_server_submit(vof_server *S, vof_mesh *mesh, const double *alpha0,
                             const double *U0c, const double *F0, int32_t n_steps,
                             const double *dt, const double *scale, vof_job **job) {
  if (!S || !mesh || !alpha0 || !U0c || !F0 || !dt || !scale || !job)
    return fail(VOF_EINVAL, "null argument");
  *job = nullptr;
  if (n_steps < 1) return fail(VOF_EINVAL, "a job advects at least one step");
  if (mesh->ctx->device != S->ctx.device) return fail(VOF_EINVAL, "mesh on another device");
  if (mesh->dp.wisps || mesh->dp.band || mesh->dp.check_stencil)
    return fail(VOF_EINVAL, "jobs run without wisps, narrow band and stencil check");
  for (int32_t i = 0; i < n_steps; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i]) || !std::isfinite(scale[i]))
      return fail(VOF_EINVAL, "dt must be positive and finite, scale finite (step %d)", i);
  const DMesh &m = mesh->dm;
  vof_job *j = new (std::nothrow) vof_job;
  if (!j) return fail(VOF_ENOMEM, "host allocation failed");
  j->srv = S;
  j->mesh = mesh;
  j->steps = n_steps;
  j->L = state_layout(m, n_steps);
  if (j->L.bytes > S->arena.size) {
    delete j;
    return fail(VOF_EBUSY, "job needs %zu bytes of state, above the budget of %zu",
                j->L.bytes, S->arena.size);
  }
  j->alpha0.assign(alpha0, alpha0 + m.nc);
  j->U0c.assign(U0c, U0c + 3 * m.nc);
  j->F0.assign(F0, F0 + m.nf);
  j->dt.assign(dt, dt + n_steps);
  j->sc.assign(scale, scale + n_steps);
  for (int64_t f = 0; f < m.nf; ++f) j->nflux += F0[f] != 0.0;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    if (S->error) {
      delete j;
      return fail(S->error, "server stopped: %s", S->error_msg.c_str());
    }
    if (S->pending.size() >= 4096) {
      delete j;
      return fail(VOF_EBUSY, "the server's queue is full");
    }
    j->t_arrive = now_s();
    if (S->t_first_arrival < 0) S->t_first_arrival = j->t_arrive;
    S->pending.push_back(j);
  }
  S->cv_work.notify_one();
  *job = j;
  return VOF_OK;
}

vof_status vof_server_wait(vof_job *j, double *alpha_out, double *latency_s) {
  if (!j) return fail(VOF_EINVAL, "null argument");
  vof_server *S = j->srv;
  {
    std::unique_lock<std::mutex> lock(S->mu);
    S->cv_done.wait(lock, [&] { return j->state == kDone || S->error != VOF_OK; });
    if (j->state != kDone) return fail(S->error, "server stopped: %s", S->error_msg.c_str());
  }
  if (alpha_out) std::memcpy(alpha_out, j->h_out, 8 * (size_t)j->mesh->dm.nc);
  if (latency_s) *latency_s = j->t_done - j->t_arrive;
  vof_status rc = j->status;
  (void)hipHostFree(j->h_out);
  (void)hipEventDestroy(j->ev);
  delete j;
  if (rc) return fail(rc, "a clipped polytope exceeded its capacity");
  return VOF_OK;
}

vof_status vof_server_get_stats(vof_server *S, vof_server_stats *out) {
  if (!S || !out) return fail(VOF_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(S->mu);
  out->jobs_done = S->jobs_done;
  out->jobs_waiting = (int64_t)S->pending.size();
  out->face_fluxes = S->face_fluxes;
  out->ticks = S->ticks;
  out->latency_p50_s = percentile(S->latencies, 0.50);
  out->latency_p99_s = percentile(S->latencies, 0.99);
  out->latency_max_s = S->latencies.empty() ? 0.0
                                            : *std::max_element(S->latencies.begin(),
                                                                S->latencies.end());
  const double span = S->t_first_arrival < 0 ? 0.0 : S->t_last_done - S->t_first_arrival;
  out->face_fluxes_per_s = span > 0 ? (double)S->face_fluxes / span : 0.0;
  out->max_resident = S->max_resident;
  out->budget_bytes = (int64_t)S->arena.size;
  out->peak_bytes = (int64_t)S->arena.peak;
  return S->error;
}

vof_status vof_server_destroy(vof_server *S) {
  if (!S) return VOF_OK;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ctx.device);
  (void)hipStreamSynchronize(S->stream);
  // jobs never waited for
  for (vof_job *j : S->draining) {
    (void)hipHostFree(j->h_out);
    (void)hipEventDestroy(j->ev);
    delete j;
  }
  for (vof_job *j : S->resident) {
    (void)hipHostFree(j->h_out);
    (void)hipEventDestroy(j->ev);
    delete j;
  }
  for (vof_job *j : S->pending) delete j;
  for (auto &e : S->tick_ev)
    if (e) (void)hipEventDestroy(e);
  char *arena = S->arena_base;
  hipStream_t st = S->stream;
  delete S;  // the batch core first (its graphs and table)
  if (arena) (void)hipFree(arena);
  if (st) (void)hipStreamDestroy(st);
  return VOF_OK;
}

}  // extern "C"
