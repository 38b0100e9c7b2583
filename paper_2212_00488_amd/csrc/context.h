// Host-side state shared by the library's sources: the context behind the
// opaque stereo_ctx handle, error reporting and scratch carving.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "stereo.h"

namespace stereo_host {
struct Plan;      // plan of the integer path, per (W, H, Dmax, params)
struct SoftPlan;  // plan of the soft-argmin head, per (n, W, H, Dmax, params)
void free_soft_plans(std::vector<SoftPlan*>& plans);
}  // namespace stereo_host

namespace stereo_host {
// d-chunk size (disparities) for groups x D of work over band rows of height
// rows, from the model of the per-XCD dispatch queues (stereo.hip).
int best_chunk_size(int groups, int D, int rows, int num_cu);

// A launch geometry chosen by stereo_autotune for one shape and parameter set.
struct Tuned {
  int W, H, Dmax, npair;
  stereo_params p;
  int csize;  // disparities per k_match d-chunk
};
}  // namespace stereo_host

struct stereo_ctx {
  int device = 0;
  // stage timing: one set of STEREO_NUM_STAGES + 1 events per timed call
  std::vector<hipEvent_t> events;
  int timed_calls = 0;
  int num_cu = 256;
  size_t mem_cap = 0, used = 0;
  std::vector<stereo_host::Plan*> plans;
  std::vector<stereo_host::SoftPlan*> soft_plans;
  std::string err;
  stereo_host::Plan* last = nullptr;  // plan of the last call that kept its intermediates
  uint64_t tick = 0;
  std::vector<stereo_host::Tuned> tuned;  // d-chunk sizes chosen by stereo_autotune
  // scratch of the L1 loss entry points, one block per stream
  std::vector<std::pair<hipStream_t, void*>> l1_blocks;
  // device address of this device's fixed scratch array (stereo_disparity_noalloc),
  // or null with the reason in noalloc_err
  void* noalloc_scratch = nullptr;
  std::string noalloc_err;
};

namespace stereo_host {

inline int fail(stereo_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return stereo_host::fail(ctx, STEREO_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <class T>
T* carve(char*& cur, size_t count) {
  T* p = reinterpret_cast<T*>(cur);
  cur += (count * sizeof(T) + 255) & ~size_t(255);
  return p;
}

}  // namespace stereo_host
