// vof_host_internal.h -- host-side objects shared by the library's host
// sources (the C ABI's opaque structs, error reporting).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/vof.h"
#include "vof_internal.h"

namespace vof {
// Record a description of the failure for vof_last_error() and return code.
vof_status fail(vof_status code, const char *fmt, ...);
const char *last_error();
// latched device flags (read after a synchronisation) -> status
vof_status flags_status(const uint32_t *d_flags);
}  // namespace vof

#define HIP_OR_FAIL(expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return ::vof::fail(VOF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct vof_context {
  int device;
  hipStream_t stream;
};

struct vof_mesh {
  vof_context *ctx = nullptr;  // copy of the creating context (device, stream)
  vof::DMesh dm{};
  vof::DState ds{};
  vof::DParams dp{};
  std::vector<void *> allocs;
  int64_t bytes = 0;
  int32_t max_cell_faces = 0;
  int64_t st_entries = 0;
  int64_t step_cap = 0;
  vof_context own_ctx{};
  bool have_alpha = false, have_velocity = false;
  double *stats_buf = nullptr;  // 4 doubles
  bool profiling = false;
  vof::Prof prof;
  // the launch sequence of one step captured once (valid while the kernel
  // arguments -- buffers and parameters -- stay as captured)
  hipStream_t cap_stream = nullptr;
  vof::Fork fork;  // side stream and events of the captured step
  hipGraphExec_t step_graph = nullptr;
  bool graph_ok = false;
  double prof_ms[vof::kKNum] = {0};
  int64_t prof_count[vof::kKNum] = {0};

  template <class T>
  vof_status alloc(T **p, int64_t count) {
    size_t nbytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, nbytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return ::vof::fail(VOF_ENOMEM, "hipMalloc of %zu bytes failed: %s", nbytes, hipGetErrorString(e));
    }
    allocs.push_back(q);
    bytes += (int64_t)nbytes;
    *p = (T *)q;
    return VOF_OK;
  }
  ~vof_mesh() {
    if (step_graph) (void)hipGraphExecDestroy(step_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (fork.side) (void)hipStreamDestroy(fork.side);
    if (fork.fork) (void)hipEventDestroy(fork.fork);
    if (fork.join) (void)hipEventDestroy(fork.join);
    for (int i = 0; i < prof.cap; ++i) {
      (void)hipEventDestroy(prof.recs[i].a);
      (void)hipEventDestroy(prof.recs[i].b);
    }
    delete[] prof.recs;
    for (void *q : allocs) (void)hipFree(q);
  }
};

