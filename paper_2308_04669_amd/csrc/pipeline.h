// Shared device-side state of the depth / shading / shadow pipeline: pair
// lists in the workspace, kernel arguments and small epilogue helpers.
#pragma once
#include "device_common.h"
#include "launch.h"
#include "mlp_engine.h"

namespace nedf {

// Kernel arguments shared by the stages (passed by value).
struct KArgs {
  RaySrc rays;
  int64_t n_rays;
  int32_t n_obj, n_inst;
  ObjDesc obj[NEDF_MAX_OBJECTS];
  const int32_t* inst_object;
  const float* w2l;
  // instance index written into the depth keys (null: the scene's own
  // index); lets keys of a subset of a scene carry the full scene's indices
  const int32_t* inst_gid;
  int32_t n_samples, clip;
  float t_near, t_far, hit_thr;
  uint32_t item_mask;    // objects whose pairs the matrix-core stage takes
  int32_t item_pairs;    // pairs per work item of that stage
  int* status;
  WsCounters* C;
  PairList* L;           // list the current stage reads
  uint2* pairs;          // its pair array
  PairList* LB;          // second list (fallback)
  uint2* pairsB;
  uint2* pairsS;         // depth-slab list of the network stage
  float* pair_dm;        // per pair of list A: lowest depth it can report (world units)
  uint8_t* pair_slab;    // per pair of list A: its depth slab (network stage)
  uint32_t* slab_mask;   // per SLAB_BLOCK pairs of list A: bit s set if slab s occurs
  // shadow-ray queries: only whether some hit lies closer than
  // ray_tmax[ray] - tmax_eps matters (null for depth queries)
  const float* ray_tmax;
  float tmax_eps;
  // ray arrays laid out as an image of this width (shadow rays, one per
  // pixel): culled in 16 x 16 tiles; 0 for unstructured arrays
  int32_t ray_grid_w;
  int64_t capacity;
  uint64_t* keys;
  uint32_t* opac;
  float* depth;
  int32_t* id;
  float* opacity;
  // NeDF inference
  float p_lo, p_hi;
  // refinement / shading / shadow
  float refine_h;
  int32_t refine_steps;
  int32_t shade_K;
  float shade_h;
  float rs_sigma;       // outlier threshold of deferred shading (0: off)
  int32_t shade_chord;  // second pass: samples over the bounding chord of list B's pixels
  float clear_rgb[3];
  float* rgb;
};

// Depth beyond which a pair of `ray` can no longer change the result: the
// pixel's nearest hit so far; for shadow queries the occlusion distance, or
// -inf once the ray is already known to be occluded.
__device__ __forceinline__ float depth_limit(const KArgs& a, uint32_t ray) {
  const float best = __uint_as_float(uint32_t(a.keys[ray] >> 32));
  if (!a.ray_tmax) return best;
  const float cut = a.ray_tmax[ray] - a.tmax_eps;
  return best < cut ? -INFINITY : cut;
}

__device__ __forceinline__ void neu_add(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

__device__ __forceinline__ float analytic_sigma(const ObjDesc& od, float x, float y, float z) {
  if (od.field == NEDF_FIELD_SPHERE) {
    const float r = sqrtf(x * x + y * y + z * z);
    return od.param[0] * sigmoidf_((od.param[1] - r) / od.param[2]);
  }
  return (z >= od.param[1] && z <= od.param[2]) ? od.param[0] : 0.0f;
}

// Density of an MLP field from the raw head output u at local point x.
__device__ __forceinline__ float mlp_sigma(const ObjDesc& od, float u, float x, float y, float z) {
  if (od.sigma_mode == NEDF_SIGMA_SDF)
    return od.param[0] * sigmoidf_(u - sdf_shape(int(od.param[2]), x, y, z) / od.param[1]);
  const float s = softplusf_(u);
  if (od.sigma_mode == NEDF_SIGMA_SOFTPLUS_MASKED)
    return (x * x + y * y + z * z <= od.bound * od.bound) ? s : 0.0f;
  return s;
}

// Surface function (logit of sigma / sigma_max) of an SDF-mode MLP field.
__device__ __forceinline__ float mlp_surface(const ObjDesc& od, float u, float x, float y, float z) {
  return u - sdf_shape(int(od.param[2]), x, y, z) / od.param[1];
}

__device__ __forceinline__ void emit_key(const KArgs& a, uint32_t ray, uint32_t inst, float D) {
  const int gid = a.inst_gid ? a.inst_gid[inst] : int(inst);
  atomicMin(reinterpret_cast<unsigned long long*>(&a.keys[ray]), (unsigned long long)pack_key(D, gid));
}

// Work item -> (object, first pair) of list L (items of `per` pairs).
__device__ __forceinline__ int item_object(const PairList* L, int n_obj, int item) {
  int obj = 0;
  while (obj + 1 < n_obj && L->item_start[obj + 1] <= item) ++obj;
  return obj;
}

}  // namespace nedf
