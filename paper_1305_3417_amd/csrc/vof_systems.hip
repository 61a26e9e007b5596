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
  // captured step per kinds mask (0..7), valid for `conf`
  hipStream_t cap_stream = nullptr;
  Fork fork;
  hipGraphExec_t graph[8] = {nullptr};
  BConf graph_conf[8];

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
