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

// A per-object list of (ray or pixel, instance) pairs in the workspace:
// object m owns pairs[off[m] .. off[m] + cnt[m]); item_start is the prefix of
// work items over the objects a stage processes.
struct PairList {
  int32_t cnt[NEDF_MAX_OBJECTS];
  int32_t fill[NEDF_MAX_OBJECTS];
  int32_t off[NEDF_MAX_OBJECTS + 1];
  int32_t item_start[NEDF_MAX_OBJECTS + 1];
  int32_t total_items, work_counter, total_pairs, pad;
};

// Device counters in the workspace (after the 256-byte status block).
struct WsCounters {
  PairList A;       // primary pairs (culling result) / binned pixels
  PairList B;       // fallback pairs (NeDF uncertain rays)
  PairList S;       // pairs of the current depth slab of the network stage
  int32_t stats[8]; // [0] pairs decided by the network, [1] sent to the marcher, [2] network misses,
                    // [3] marcher pairs left after the depth test, [4] pairs after culling
  uint32_t dmin_bits, dmax_bits;  // range of the pairs' lowest possible depths (float bits, >= 0)
};

// Workspace layout: status | counters | keys | opacity bits | extra (shadow
// rays) | pairs A | pairs B | pairs S | depth bounds of list A | depth slabs
// of list A | per 1024 pairs of list A, the set of slabs present (one bit per
// slab).  Capacity is per pair list (a multiple of SLAB_BLOCK).
constexpr size_t WS_BYTES_PER_PAIR = 3 * 8 + 4 + 1;
constexpr int SLAB_BLOCK = 1024;
struct WsLayout {
  size_t counters, keys, opac, pairs, pairsB, pairsS, pairsD, pairsSlab, slabMask, extra, end;
  int64_t capacity;
};

WsLayout ws_layout(int64_t n_rays, size_t extra_bytes, size_t ws_bytes);
size_t ws_fixed_bytes(int64_t n_rays, size_t extra_bytes);

hipError_t launch_compose_transforms(const double* G, int32_t n, float* w2l, hipStream_t s);

bool march_mlp_supported(int dtype, int width, int n_hidden, int L);
// Waves per workgroup of the marcher launch the tuning table selects (the
// pairs per work item of a list it marches).
int march_waves(int dtype, int width);
bool nedf_net_supported(int dtype, int width, int n_hidden, int L);
bool shade_supported(int dtype, const nedf_mlp_shape& s);
bool refine_supported(int dtype, const nedf_mlp_shape& s);

struct KArgs;

// Stages (kernels enqueued on s, no host synchronisation).
void stage_init_cull(const KArgs& k, hipStream_t s, uint32_t item_mask, int item_pairs);
void stage_march(const KArgs& k, hipStream_t s, bool list_b, uint32_t analytic_mask, int dtype, int W, int H,
                 int L);
// Intersection-network stage over list A, front to back in n_slabs depth
// slabs (objects in nedf_mask).
void stage_nedf(const KArgs& k, hipStream_t s, int dtype, uint32_t nedf_mask, int n_slabs,
                bool classifier = false);
// Classifier-form networks (NEDF_IN_POINTS16) over the current slab list.
void launch_nedf_cls(const KArgs& k, hipStream_t s, int dtype);
bool nedf_cls_supported(int dtype, const nedf_mlp_shape& s);
void stage_finalize(const KArgs& k, hipStream_t s);
constexpr int MAX_KEY_SETS = 8;
struct KeySets {
  const uint64_t* p[MAX_KEY_SETS];
  int32_t n;
};
void stage_merge_keys(const KArgs& k, hipStream_t s, const KeySets& ks);
void stage_bin_pixels(const KArgs& k, hipStream_t s, const int32_t* ids, uint32_t mask, int per);
void stage_refine(const KArgs& k, hipStream_t s, const int32_t* ids, uint32_t mlp_mask, uint32_t sphere_mask,
                  int dtype);
// rs_samples > 0: pixels whose density stays below k.rs_sigma at every one of
// their K samples are shaded again by volume rendering over the bounding
// chord with rs_samples samples.
void stage_shade(const KArgs& k, hipStream_t s, const int32_t* ids, uint32_t nerf_mask, int dtype,
                 int rs_samples = 0);
void stage_shadow_rays(const KArgs& k, hipStream_t s, const int32_t* ids, const float L[3], float dir_dist, float* so,
                       float* sd, float* dist);
void stage_shadow_init(const KArgs& k, hipStream_t s, float* shadow);
void stage_shadow_apply(const KArgs& k, hipStream_t s, const int32_t* ids, const float* depth_l, const float* dist,
                        float eps, float beta, float* shadow);
void stage_composite(const KArgs& k, hipStream_t s, const float* shadow, float* rgb);

size_t train_ws_bytes(const nedf_mlp_shape& sh, int B);
hipError_t launch_train_init(const nedf_mlp_shape& sh, const float* const* W, const float* const* b, uint8_t* st,
                             hipStream_t s);
hipError_t launch_train_step(const nedf_mlp_shape& sh, uint8_t* st, const float* o_l, const float* d_l,
                             const float* depth, const uint8_t* hit, int B, float lr, float b1, float b2, float eps,
                             float w_hit, float bound, float* loss, uint8_t* ws, hipStream_t s);
hipError_t launch_fp8_calibrate(const nedf_mlp_shape& sh, const float* const* W, const float* const* b,
                                const float* o_l, const float* d_l, int B, float* scales, uint8_t* ws,
                                hipStream_t s);
size_t fp8_calibrate_ws_bytes(const nedf_mlp_shape& sh, int B);
hipError_t launch_train_export(const nedf_mlp_shape& sh, const uint8_t* st, float* const* W, float* const* b,
                               bool grads, hipStream_t s);

}  // namespace nedf
