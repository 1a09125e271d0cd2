// Host-side launch interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nedf.h"

namespace nedf {

// Per-object description passed to kernels by value.
struct ObjDesc {
  int32_t field, sigma_mode;
  float bound;
  float param[6];
  const uint8_t* blob;      // density network blob (device) or NULL
  const uint8_t* nedf_blob; // intersection network blob (device) or NULL
};

struct RaySrcHost {
  int32_t kind, width, height;
  float eye[3], fwd[3], right[3], up[3];
  const float* o;
  const float* d;
  int64_t n;
};

// Device counters in the workspace (after the 256-byte status block).
struct WsCounters {
  int32_t cnt[NEDF_MAX_OBJECTS];
  int32_t fill[NEDF_MAX_OBJECTS];
  int32_t off[NEDF_MAX_OBJECTS + 1];
  int32_t item_start[NEDF_MAX_OBJECTS + 1];
  int32_t total_items, work_counter, total_pairs, capacity;
};

struct WsLayout {
  size_t counters, keys, opac, pairs, end;
  int64_t capacity;
};

WsLayout ws_layout(int64_t n_rays, size_t ws_bytes);
size_t ws_fixed_bytes(int64_t n_rays);

struct MarchLaunch {
  RaySrcHost rays;
  int32_t n_obj, n_inst;
  ObjDesc obj[NEDF_MAX_OBJECTS];
  const int32_t* inst_object;
  const float* inst_w2l;
  int32_t n_samples, clip;
  float t_near, t_far, hit_thr;
  int32_t dtype;
  int32_t mlp_width, mlp_hidden, mlp_L;  // shared shape of all MLP objects (0 if none)
  uint8_t* ws;
  WsLayout lay;
  float* depth;
  int32_t* id;
  float* opacity;
};

hipError_t launch_compose_transforms(const double* G, int32_t n, float* w2l, hipStream_t s);
hipError_t launch_march(const MarchLaunch& a, hipStream_t s);
bool march_mlp_supported(int dtype, int width, int n_hidden, int L);

}  // namespace nedf
