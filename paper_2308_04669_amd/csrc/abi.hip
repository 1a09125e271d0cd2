// C-ABI entry points: argument validation, workspace planning and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "blob_layout.h"
#include "launch.h"
#include "nedf.h"
#include "pipeline.h"
#include "runtime.h"
#include "train_layout.h"

namespace nedf {

namespace {
thread_local std::string g_last_error;

__global__ void k_reset_status(int* status) {
  if (threadIdx.x == 0) *status = 0;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int64_t ray_count(const nedf_rays* r) {
  if (!r) return -1;
  if (r->kind == 0) return int64_t(r->camera.width) * int64_t(r->camera.height);
  return r->n;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {
struct ProfRec {
  std::string name;  // "outer/inner" for stages nested in another stage
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
std::map<const void*, std::vector<size_t>> g_prof_open;  // stream -> stack of open records

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

// Set while a fixed-memory entry point runs on this thread: it records no
// profiling events (creating them could allocate).
thread_local bool g_prof_suppress = false;

bool prof_on() { return g_prof_on && !g_prof_suppress; }

void prof_mark(const char* name, void* stream, bool begin) {
  if (!g_prof_on || g_prof_suppress) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<size_t>& open = g_prof_open[stream];
  if (begin) {
    ProfRec r{open.empty() ? std::string(name) : g_prof_recs[open.back()].name + "/" + name, prof_event(),
              prof_event()};
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, s);
    open.push_back(g_prof_recs.size());
    g_prof_recs.push_back(r);
  } else {
    if (open.empty()) return;
    (void)hipEventRecord(g_prof_recs[open.back()].b, s);
    open.pop_back();
  }
}

int32_t fail(int32_t code, const std::string& msg) {
  g_last_error = msg;
  return code;
}


// Workspace: status(256) | counters | keys n*8 | opacity n*4 | extra | pairs A | B | S | depth bounds.
size_t ws_fixed_bytes(int64_t n_rays, size_t extra_bytes) {
  size_t off = 256;
  off = align256(off + sizeof(WsCounters));
  off = align256(off + size_t(n_rays) * 8);
  off = align256(off + size_t(n_rays) * 4);
  off = align256(off + extra_bytes);
  return off;
}

WsLayout ws_layout(int64_t n_rays, size_t extra_bytes, size_t ws_bytes) {
  WsLayout l;
  l.counters = 256;
  l.keys = align256(l.counters + sizeof(WsCounters));
  l.opac = align256(l.keys + size_t(n_rays) * 8);
  l.extra = align256(l.opac + size_t(n_rays) * 4);
  l.pairs = align256(l.extra + extra_bytes);
  // per pair WS_BYTES_PER_PAIR, plus 4 bytes per SLAB_BLOCK pairs, plus slack
  const int64_t avail = ws_bytes > l.pairs + 1024 ? int64_t(ws_bytes - l.pairs - 1024) : 0;
  int64_t cap = avail / int64_t(WS_BYTES_PER_PAIR * SLAB_BLOCK + 4) * SLAB_BLOCK;
  if (cap > (int64_t(1) << 31) - SLAB_BLOCK) cap = (int64_t(1) << 31) - SLAB_BLOCK;
  l.capacity = cap;
  l.pairsB = l.pairs + size_t(cap) * 8;
  l.pairsS = l.pairsB + size_t(cap) * 8;
  l.pairsD = l.pairsS + size_t(cap) * 8;
  l.pairsSlab = l.pairsD + size_t(cap) * 4;
  l.slabMask = l.pairsSlab + size_t(cap);
  l.end = l.slabMask + size_t(cap / SLAB_BLOCK) * 4;
  return l;
}

namespace {

constexpr size_t SHADOW_EXTRA_PER_RAY = 32;  // origin 12 + direction 12 + distance 4 + depth 4

int32_t check_rays(const nedf_rays* rays, RaySrcHost& rs) {
  if (!rays) return fail(NEDF_ERR_NULL, "rays is NULL");
  std::memset(&rs, 0, sizeof(rs));
  rs.kind = rays->kind;
  if (rays->kind == 0) {
    const nedf_camera& c = rays->camera;
    if (c.width <= 0 || c.height <= 0) return fail(NEDF_ERR_SHAPE, "camera width/height must be positive");
    if (!(c.fov_y_deg > 0.0 && c.fov_y_deg < 180.0)) return fail(NEDF_ERR_SHAPE, "camera fov must be in (0, 180)");
    double f[3] = {c.at[0] - c.eye[0], c.at[1] - c.eye[1], c.at[2] - c.eye[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(NEDF_ERR_SHAPE, "camera eye equals at");
    for (double& v : f) v /= fl;
    double r[3] = {f[1] * c.up[2] - f[2] * c.up[1], f[2] * c.up[0] - f[0] * c.up[2], f[0] * c.up[1] - f[1] * c.up[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0.0)) return fail(NEDF_ERR_SHAPE, "camera up is parallel to the view direction");
    for (double& v : r) v /= rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double th = std::tan(c.fov_y_deg * M_PI / 360.0);
    const double aspect = double(c.width) / double(c.height);
    for (int i = 0; i < 3; ++i) {
      rs.eye[i] = float(c.eye[i]);
      rs.fwd[i] = float(f[i]);
      rs.right[i] = float(r[i] * th * aspect);
      rs.up[i] = float(u[i] * th);
    }
    rs.width = c.width;
    rs.height = c.height;
    rs.n = int64_t(c.width) * c.height;
  } else if (rays->kind == 1) {
    if (rays->n < 0) return fail(NEDF_ERR_SHAPE, "ray count is negative");
    if (rays->n > 0 && (!rays->origins || !rays->dirs)) return fail(NEDF_ERR_NULL, "ray arrays are NULL");
    if (!aligned16(rays->origins) || !aligned16(rays->dirs)) return fail(NEDF_ERR_ALIGN, "ray arrays must be 16-byte aligned");
    rs.o = rays->origins;
    rs.d = rays->dirs;
    rs.n = rays->n;
  } else {
    return fail(NEDF_ERR_SHAPE, "rays.kind must be 0 (camera) or 1 (arrays)");
  }
  if (rs.n > (int64_t(1) << 31) - 1) return fail(NEDF_ERR_SHAPE, "too many rays (limit 2^31 - 1)");
  return NEDF_OK;
}

int32_t hip_fail(hipError_t e, const char* where) {
  return fail(NEDF_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Validated scene: object descriptors, per-kind masks and the shared
// network shapes of the kernels that will run.
struct Prepared {
  KArgs k;
  int32_t nedf_dtype = -1;            // precision of the intersection networks
  uint32_t analytic = 0, mlp = 0, nedf = 0, sphere = 0, sdf_mlp = 0, nerf = 0;
  bool nedf_cls = false;  // intersection networks in the classifier form
  int32_t W = 0, H = 0, L = 0;        // density network shape (0 if none)
  nedf_mlp_shape dshape{};
};

int32_t prepare_scene(const nedf_scene* sc, int32_t dtype, Prepared& P) {
  if (!sc) return fail(NEDF_ERR_NULL, "scene is NULL");
  if (sc->n_objects < 1 || sc->n_objects > NEDF_MAX_OBJECTS) return fail(NEDF_ERR_SHAPE, "n_objects must be 1..32");
  if (!sc->objects) return fail(NEDF_ERR_NULL, "scene.objects is NULL");
  if (sc->n_inst < 1) return fail(NEDF_ERR_SHAPE, "n_inst must be >= 1");
  if (!sc->inst_object || !sc->inst_w2l) return fail(NEDF_ERR_NULL, "instance arrays are NULL");
  if (!aligned16(sc->inst_object) || !aligned16(sc->inst_w2l)) return fail(NEDF_ERR_ALIGN, "instance arrays must be 16-byte aligned");
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return fail(NEDF_ERR_DTYPE, "dtype must be F32 or BF16");
  std::memset(&P.k, 0, sizeof(P.k));
  P.k.n_obj = sc->n_objects;
  P.k.n_inst = sc->n_inst;
  P.k.inst_object = sc->inst_object;
  P.k.w2l = sc->inst_w2l;
  bool have = false;
  for (int i = 0; i < sc->n_objects; ++i) {
    const nedf_object& o = sc->objects[i];
    ObjDesc& d = P.k.obj[i];
    if (!(o.bound > 0.0f)) return fail(NEDF_ERR_SHAPE, "object bound must be positive");
    if (o.field < NEDF_FIELD_SPHERE || o.field > NEDF_FIELD_MLP) return fail(NEDF_ERR_SHAPE, "unknown object field");
    d.field = o.field;
    d.sigma_mode = o.sigma_mode;
    d.bound = o.bound;
    for (int j = 0; j < 6; ++j) d.param[j] = o.param[j];
    d.blob = static_cast<const uint8_t*>(o.density.blob);
    d.nedf_blob = static_cast<const uint8_t*>(o.nedf.blob);
    if (o.field == NEDF_FIELD_SPHERE) {
      if (!(o.param[2] > 0.0f)) return fail(NEDF_ERR_SHAPE, "sphere width must be positive");
      P.sphere |= 1u << i;
    }
    if (o.field != NEDF_FIELD_MLP) P.analytic |= 1u << i;
    if (o.field == NEDF_FIELD_MLP) {
      const nedf_mlp_shape& s = o.density.shape;
      if (!o.density.blob) return fail(NEDF_ERR_NULL, "MLP object without a density blob");
      if (!aligned16(o.density.blob)) return fail(NEDF_ERR_ALIGN, "density blob must be 16-byte aligned");
      if (o.sigma_mode < NEDF_SIGMA_SOFTPLUS || o.sigma_mode > NEDF_SIGMA_SDF) return fail(NEDF_ERR_SHAPE, "unknown sigma mode");
      if (o.sigma_mode == NEDF_SIGMA_SDF && !(o.param[1] > 0.0f)) return fail(NEDF_ERR_SHAPE, "sdf width must be positive");
      if (s.in_kind != NEDF_IN_XYZ || s.n_out != 1) return fail(NEDF_ERR_SHAPE, "density network must take xyz and output one value");
      if (o.density.dtype != dtype) return fail(NEDF_ERR_DTYPE, "density blob dtype differs from the call's dtype");
      if (!march_mlp_supported(dtype, s.width, s.n_hidden, s.enc_L))
        return fail(NEDF_ERR_UNSUPPORTED, "density network shape not instantiated (width 64/3 hidden/L6 or 256/8/L10)");
      if (have && (s.width != P.W || s.n_hidden != P.H || s.enc_L != P.L))
        return fail(NEDF_ERR_UNSUPPORTED, "all MLP objects of one call must share a network shape");
      have = true;
      P.W = s.width;
      P.H = s.n_hidden;
      P.L = s.enc_L;
      P.dshape = s;
      P.mlp |= 1u << i;
      if (o.sigma_mode == NEDF_SIGMA_SDF) P.sdf_mlp |= 1u << i;
      if (s.rgb_width > 0) P.nerf |= 1u << i;
    }
    if (o.nedf.blob) {
      const nedf_mlp_shape& s = o.nedf.shape;
      if (!aligned16(o.nedf.blob)) return fail(NEDF_ERR_ALIGN, "intersection network blob must be 16-byte aligned");
      const bool cls = s.in_kind == NEDF_IN_POINTS16;
      if (!cls && (s.in_kind != NEDF_IN_PLUECKER || s.n_out != 2))
        return fail(NEDF_ERR_SHAPE, "intersection network must take Pluecker coordinates and output (mu, logit), "
                                    "or be a classifier-form network");
      if (o.nedf.dtype != dtype && o.nedf.dtype != NEDF_FP8 && o.nedf.dtype != NEDF_FP8_MX)
        return fail(NEDF_ERR_DTYPE, "intersection network dtype must be the call's dtype, FP8 or FP8_MX");
      if (cls && o.nedf.dtype == NEDF_FP8_MX)
        return fail(NEDF_ERR_UNSUPPORTED, "MX FP8 covers the regression-form network");
      if (P.nedf_dtype >= 0 && o.nedf.dtype != P.nedf_dtype)
        return fail(NEDF_ERR_UNSUPPORTED, "all intersection networks of one call must share a dtype");
      if (P.nedf && cls != P.nedf_cls)
        return fail(NEDF_ERR_UNSUPPORTED, "all intersection networks of one call must share a form");
      P.nedf_dtype = o.nedf.dtype;
      P.nedf_cls = cls;
      if (cls ? !nedf_cls_supported(o.nedf.dtype, s) : !nedf_net_supported(o.nedf.dtype, s.width, s.n_hidden, s.enc_L))
        return fail(NEDF_ERR_UNSUPPORTED, cls ? "classifier network not instantiated (F32/BF16, width 256, L10, "
                                                "1..64 blocks, 193 outputs)"
                                              : "intersection network shape not instantiated (width 256, 8 hidden, L8)");
      P.nedf |= 1u << i;
    }
  }
  return NEDF_OK;
}

int32_t prepare_ws(Prepared& P, const RaySrcHost& rs, size_t extra, void* ws, size_t ws_bytes, WsLayout& lay) {
  if (!ws) return fail(NEDF_ERR_NULL, "workspace is NULL");
  if (!aligned16(ws)) return fail(NEDF_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (ws_bytes < ws_fixed_bytes(rs.n, extra) + 16) return fail(NEDF_ERR_WORKSPACE, "workspace smaller than nedf_workspace_size()");
  lay = ws_layout(rs.n, extra, ws_bytes);
  uint8_t* w = static_cast<uint8_t*>(ws);
  KArgs& k = P.k;
  k.status = reinterpret_cast<int*>(w);
  k.C = reinterpret_cast<WsCounters*>(w + lay.counters);
  k.keys = reinterpret_cast<uint64_t*>(w + lay.keys);
  k.opac = reinterpret_cast<uint32_t*>(w + lay.opac);
  k.pairs = reinterpret_cast<uint2*>(w + lay.pairs);
  k.pairsB = reinterpret_cast<uint2*>(w + lay.pairsB);
  k.pairsS = reinterpret_cast<uint2*>(w + lay.pairsS);
  k.pair_dm = reinterpret_cast<float*>(w + lay.pairsD);
  k.pair_slab = w + lay.pairsSlab;
  k.slab_mask = reinterpret_cast<uint32_t*>(w + lay.slabMask);
  k.capacity = lay.capacity;
  return NEDF_OK;
}

void set_rays(KArgs& k, const RaySrcHost& rs) {
  k.rays.kind = rs.kind;
  k.rays.width = rs.width;
  k.rays.height = rs.height;
  for (int i = 0; i < 3; ++i) {
    k.rays.eye[i] = rs.eye[i];
    k.rays.fwd[i] = rs.fwd[i];
    k.rays.right[i] = rs.right[i];
    k.rays.up[i] = rs.up[i];
  }
  k.rays.o = rs.o;
  k.rays.d = rs.d;
  k.n_rays = rs.n;
}

int32_t check_march_opts(const nedf_march_opts* o) {
  if (!o) return fail(NEDF_ERR_NULL, "march opts are NULL");
  if (o->n_samples < 1 || o->n_samples > 4096) return fail(NEDF_ERR_SHAPE, "n_samples must be 1..4096");
  if (!(o->hit_threshold > 0.0f && o->hit_threshold <= 1.0f)) return fail(NEDF_ERR_SHAPE, "hit_threshold must be in (0, 1]");
  if (!o->clip_to_bound && !(o->t_far > o->t_near && o->t_near >= 0.0f)) return fail(NEDF_ERR_SHAPE, "need 0 <= t_near < t_far");
  return NEDF_OK;
}

int32_t check_infer_opts(const nedf_infer_opts* o) {
  if (!o) return fail(NEDF_ERR_NULL, "infer opts are NULL");
  if (!(o->p_lo >= 0.0f && o->p_lo <= o->p_hi && o->p_hi <= 1.0f)) return fail(NEDF_ERR_SHAPE, "need 0 <= p_lo <= p_hi <= 1");
  if (o->refine_steps < 0 || o->refine_steps > 16) return fail(NEDF_ERR_SHAPE, "refine_steps must be 0..16");
  if (o->refine_steps > 0 && !(o->refine_h > 0.0f)) return fail(NEDF_ERR_SHAPE, "refine_h must be positive");
  int32_t st = check_march_opts(&o->march);
  if (st) return st;
  if (!o->march.clip_to_bound) return fail(NEDF_ERR_UNSUPPORTED, "fallback marching needs clip_to_bound = 1");
  return NEDF_OK;
}

void apply_march_opts(KArgs& k, const nedf_march_opts& o) {
  k.n_samples = o.n_samples;
  k.clip = o.clip_to_bound;
  k.t_near = o.t_near;
  k.t_far = o.t_far;
  k.hit_thr = o.hit_threshold;
}

// Plain-marcher depth into k.depth / k.id / k.opacity.
void run_march(const Prepared& P, int dtype, hipStream_t s) {
  stage_init_cull(P.k, s, P.mlp, march_waves(dtype, P.W));
  KArgs k = P.k;
  k.L = &k.C->A;
  stage_march(k, s, false, P.analytic, dtype, P.mlp ? P.W : 0, P.H, P.L);
  stage_finalize(P.k, s);
}

// NeDF depth keys (+ fallback) of every pair into k.keys.
void run_infer_keys(const Prepared& P, int dtype, const nedf_infer_opts& o, hipStream_t s) {
  KArgs k = P.k;
  k.p_lo = o.p_lo;
  k.p_hi = o.p_hi;
  stage_init_cull(k, s, P.nedf, 32 * eng::WAVES);
  k.L = &k.C->A;
  // analytic objects without a network are marched directly
  const uint32_t direct = P.analytic & ~P.nedf;
  if (direct) stage_march(k, s, false, direct, dtype, 0, 0, 0);
  // MX networks take the FP8 slab count
  const int slab_dt = P.nedf_dtype == NEDF_FP8_MX ? NEDF_FP8 : P.nedf_dtype;
  if (P.nedf) stage_nedf(k, s, P.nedf_dtype, P.nedf, tune_value(NEDF_TUNE_SLABS, slab_dt), P.nedf_cls);
  // uncertain pairs: marcher on list B
  stage_march(k, s, true, P.analytic, dtype, (P.mlp & P.nedf) ? P.W : 0, P.H, P.L);
}

// Keys -> depth / id, then refinement of the winners.
void run_finish(const Prepared& P, int dtype, const nedf_infer_opts& o, hipStream_t s) {
  KArgs k = P.k;
  stage_finalize(k, s);
  if (o.refine_steps > 0 && k.id) {
    k.refine_h = o.refine_h;
    k.refine_steps = o.refine_steps;
    const uint32_t mlp_ok = refine_supported(dtype, P.dshape) ? P.sdf_mlp : 0u;
    if (mlp_ok | P.sphere) stage_refine(k, s, k.id, mlp_ok, P.sphere, dtype);
  }
}

// NeDF depth (+ fallback, + refinement) into k.depth / k.id.
void run_infer(const Prepared& P, int dtype, const nedf_infer_opts& o, hipStream_t s) {
  run_infer_keys(P, dtype, o, s);
  run_finish(P, dtype, o, s);
}

}  // namespace
}  // namespace nedf

using namespace nedf;

extern "C" const char* nedf_version(void) { return "nedf-mi355x 0.2.0 (gfx950)"; }

extern "C" const char* nedf_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* nedf_status_string(int32_t s) {
  switch (s) {
    case NEDF_OK: return "ok";
    case NEDF_ERR_NULL: return "null pointer";
    case NEDF_ERR_SHAPE: return "bad shape";
    case NEDF_ERR_DTYPE: return "bad dtype";
    case NEDF_ERR_ALIGN: return "misaligned pointer";
    case NEDF_ERR_WORKSPACE: return "workspace too small";
    case NEDF_ERR_CAPACITY: return "pair capacity exceeded";
    case NEDF_ERR_HIP: return "HIP runtime error";
    case NEDF_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

extern "C" int32_t nedf_compose_transforms(const double* inst_G, int32_t n, float* inst_w2l,
                                           nedf_stream_t stream) {
  if (n < 0) return fail(NEDF_ERR_SHAPE, "nedf_compose_transforms: n < 0");
  if (n == 0) return NEDF_OK;
  if (!inst_G || !inst_w2l) return fail(NEDF_ERR_NULL, "nedf_compose_transforms: NULL argument");
  if (!aligned16(inst_G) || !aligned16(inst_w2l)) return fail(NEDF_ERR_ALIGN, "nedf_compose_transforms: misaligned");
  hipError_t e = launch_compose_transforms(inst_G, n, inst_w2l, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_compose_transforms");
  return NEDF_OK;
}

extern "C" size_t nedf_workspace_size(int32_t op, const nedf_scene* scene, const nedf_rays* rays,
                                      int64_t pair_capacity) {
  const int64_t n = ray_count(rays);
  if (n < 0 || !scene) {
    set_error("nedf_workspace_size: NULL scene or rays");
    return 0;
  }
  int64_t cap = pair_capacity > 0 ? pair_capacity : n * int64_t(scene->n_inst > 0 ? scene->n_inst : 1);
  if (cap < 1) cap = 1;
  cap = (cap + SLAB_BLOCK - 1) / SLAB_BLOCK * SLAB_BLOCK;  // the layout keeps whole slab blocks
  if (cap > (int64_t(1) << 31) - SLAB_BLOCK) cap = (int64_t(1) << 31) - SLAB_BLOCK;
  const size_t extra = op == NEDF_OP_SHADOW ? size_t(n) * SHADOW_EXTRA_PER_RAY : 0;
  return ws_fixed_bytes(n, extra) + size_t(cap) * WS_BYTES_PER_PAIR + size_t(cap / SLAB_BLOCK) * 4 + 1024;
}

extern "C" int32_t nedf_check_status(const void* ws, nedf_stream_t stream) {
  if (!ws) return fail(NEDF_ERR_NULL, "nedf_check_status: ws is NULL");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_check_status");
  int32_t st = 0;
  e = hipMemcpy(&st, ws, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "nedf_check_status");
  if (st != NEDF_OK) fail(st, "device status: pair list overflow");
  return st;
}

extern "C" int32_t nedf_ws_counters(const void* ws, nedf_stream_t stream, int64_t* out7) {
  if (!ws || !out7) return fail(NEDF_ERR_NULL, "nedf_ws_counters: NULL argument");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_ws_counters");
  WsCounters c;
  e = hipMemcpy(&c, static_cast<const uint8_t*>(ws) + 256, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "nedf_ws_counters");
  out7[0] = c.A.total_pairs;
  out7[1] = c.A.total_items;
  out7[2] = c.stats[0];
  out7[3] = c.stats[1];
  out7[4] = c.stats[2];
  out7[5] = c.stats[3];
  out7[6] = c.stats[4];
  return NEDF_OK;
}

extern "C" int32_t nedf_march_depth(const nedf_scene* scene, const nedf_rays* rays,
                                    const nedf_march_opts* opts, float* depth, int32_t* id,
                                    float* opacity, void* ws, size_t ws_bytes, nedf_stream_t stream) {
  int32_t st = check_march_opts(opts);
  if (st) return st;
  if (opts->dtype != NEDF_F32 && opts->dtype != NEDF_BF16) return fail(NEDF_ERR_DTYPE, "march dtype must be F32 or BF16");
  Prepared P;
  st = prepare_scene(scene, opts->dtype, P);
  if (st) return st;
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!depth || !id) return fail(NEDF_ERR_NULL, "depth and id are required");
  if (!aligned16(depth) || !aligned16(id) || (opacity && !aligned16(opacity)))
    return fail(NEDF_ERR_ALIGN, "output buffers must be 16-byte aligned");
  WsLayout lay;
  st = prepare_ws(P, rs, 0, ws, ws_bytes, lay);
  if (st) return st;
  set_rays(P.k, rs);
  apply_march_opts(P.k, *opts);
  P.k.depth = depth;
  P.k.id = id;
  P.k.opacity = opacity;
  hipStream_t s = static_cast<hipStream_t>(stream);
  run_march(P, opts->dtype, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "nedf_march_depth");
  return NEDF_OK;
}

namespace {
int32_t infer_impl(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts, float* depth,
                   int32_t* id, void* ws, size_t ws_bytes, nedf_stream_t stream, const char* who) {
  int32_t st = check_infer_opts(opts);
  if (st) return st;
  Prepared P;
  st = prepare_scene(scene, opts->dtype, P);
  if (st) return st;
  if (P.mlp & ~P.nedf) return fail(NEDF_ERR_UNSUPPORTED, "every MLP object needs an intersection network (use nedf_march_depth)");
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!depth || !id) return fail(NEDF_ERR_NULL, "depth and id are required");
  if (!aligned16(depth) || !aligned16(id)) return fail(NEDF_ERR_ALIGN, "output buffers must be 16-byte aligned");
  WsLayout lay;
  st = prepare_ws(P, rs, 0, ws, ws_bytes, lay);
  if (st) return st;
  set_rays(P.k, rs);
  apply_march_opts(P.k, opts->march);
  P.k.depth = depth;
  P.k.id = id;
  run_infer(P, opts->dtype, *opts, static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, who);
  return NEDF_OK;
}
}  // namespace

extern "C" int32_t nedf_infer_depth_id(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                                       float* depth, int32_t* id, void* ws, size_t ws_bytes, nedf_stream_t stream) {
  return infer_impl(scene, rays, opts, depth, id, ws, ws_bytes, stream, "nedf_infer_depth_id");
}

// ---- buffer reuse under manipulation -------------------------------------------
extern "C" int32_t nedf_infer_keys(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                                   const int32_t* inst_gid, uint64_t* keys, void* ws, size_t ws_bytes,
                                   nedf_stream_t stream) {
  int32_t st = check_infer_opts(opts);
  if (st) return st;
  Prepared P;
  st = prepare_scene(scene, opts->dtype, P);
  if (st) return st;
  if (P.mlp & ~P.nedf) return fail(NEDF_ERR_UNSUPPORTED, "every MLP object needs an intersection network (use nedf_march_depth)");
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!keys) return fail(NEDF_ERR_NULL, "nedf_infer_keys: keys is NULL");
  if (!aligned16(keys) || (inst_gid && !aligned16(inst_gid)))
    return fail(NEDF_ERR_ALIGN, "nedf_infer_keys: keys and inst_gid must be 16-byte aligned");
  WsLayout lay;
  st = prepare_ws(P, rs, 0, ws, ws_bytes, lay);
  if (st) return st;
  set_rays(P.k, rs);
  apply_march_opts(P.k, opts->march);
  P.k.inst_gid = inst_gid;
  P.k.keys = keys;  // the stages build the keys in the caller's buffer
  run_infer_keys(P, opts->dtype, *opts, static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "nedf_infer_keys");
  return NEDF_OK;
}

extern "C" int32_t nedf_compose_keys(const nedf_scene* scene, const nedf_rays* rays, const nedf_infer_opts* opts,
                                     const uint64_t* const* key_sets, int32_t n_sets, float* depth, int32_t* id,
                                     void* ws, size_t ws_bytes, nedf_stream_t stream) {
  int32_t st = check_infer_opts(opts);
  if (st) return st;
  if (n_sets < 1 || n_sets > MAX_KEY_SETS) return fail(NEDF_ERR_SHAPE, "nedf_compose_keys: n_sets must be 1..8");
  if (!key_sets) return fail(NEDF_ERR_NULL, "nedf_compose_keys: key_sets is NULL");
  KeySets ks{};
  ks.n = n_sets;
  for (int j = 0; j < n_sets; ++j) {
    if (!key_sets[j]) return fail(NEDF_ERR_NULL, "nedf_compose_keys: a key set is NULL");
    if (!aligned16(key_sets[j])) return fail(NEDF_ERR_ALIGN, "nedf_compose_keys: key sets must be 16-byte aligned");
    ks.p[j] = key_sets[j];
  }
  Prepared P;
  st = prepare_scene(scene, opts->dtype, P);
  if (st) return st;
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!depth || !id) return fail(NEDF_ERR_NULL, "depth and id are required");
  if (!aligned16(depth) || !aligned16(id)) return fail(NEDF_ERR_ALIGN, "output buffers must be 16-byte aligned");
  WsLayout lay;
  st = prepare_ws(P, rs, 0, ws, ws_bytes, lay);
  if (st) return st;
  set_rays(P.k, rs);
  apply_march_opts(P.k, opts->march);
  P.k.depth = depth;
  P.k.id = id;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, P.k.status);
  stage_merge_keys(P.k, s, ks);
  run_finish(P, opts->dtype, *opts, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "nedf_compose_keys");
  return NEDF_OK;
}

// ---- fixed-memory variant -----------------------------------------------------
// The workspace of nedf_infer_depth_id_static: a file-scope device array, one
// copy on every GPU the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel (in host code it is a
// host-side stand-in); it looks up each device's address once, with that
// device current, and uses that pointer.
constexpr size_t NEDF_STATIC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[NEDF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int32_t scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "nedf_infer_depth_id_static: hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(NEDF_ERR_UNSUPPORTED, "nedf_infer_depth_id_static: device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "nedf_infer_depth_id_static: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NEDF_OK;
}
}  // namespace

extern "C" size_t nedf_static_scratch_bytes(void) { return NEDF_STATIC_SCRATCH_BYTES; }

extern "C" int32_t nedf_infer_depth_id_static(const nedf_scene* scene, const nedf_rays* rays,
                                              const nedf_infer_opts* opts, float* depth, int32_t* id,
                                              nedf_stream_t stream) {
  if (!scene || !rays) return fail(NEDF_ERR_NULL, "nedf_infer_depth_id_static: NULL scene or rays");
  // the worst case (every ray meets every instance) must fit, so that no
  // pair list can overflow
  const size_t need = nedf_workspace_size(NEDF_OP_INFER, scene, rays, 0);
  if (need == 0) return NEDF_ERR_NULL;
  if (need > NEDF_STATIC_SCRATCH_BYTES)
    return fail(NEDF_ERR_WORKSPACE, "nedf_infer_depth_id_static: n_rays x n_instances pairs need " +
                                        std::to_string(need) + " bytes of workspace, beyond the fixed " +
                                        std::to_string(NEDF_STATIC_SCRATCH_BYTES) + " (use nedf_infer_depth_id)");
  void* ws = nullptr;
  int32_t st = scratch_of_current_device(&ws);
  if (st) return st;
  g_prof_suppress = true;
  st = infer_impl(scene, rays, opts, depth, id, ws, NEDF_STATIC_SCRATCH_BYTES, stream, "nedf_infer_depth_id_static");
  g_prof_suppress = false;
  return st;
}

extern "C" int32_t nedf_shade_deferred(const nedf_scene* scene, const nedf_rays* rays, const float* depth,
                                       const int32_t* id, const nedf_shade_opts* opts, float* rgb, void* ws,
                                       size_t ws_bytes, nedf_stream_t stream) {
  if (!opts) return fail(NEDF_ERR_NULL, "shade opts are NULL");
  const int K = opts->K;
  if (!(K == 1 || K == 2 || K == 4 || K == 8 || K == 16 || K == 32)) return fail(NEDF_ERR_SHAPE, "K must be 1, 2, 4, 8, 16 or 32");
  if (!(opts->h > 0.0f)) return fail(NEDF_ERR_SHAPE, "h must be positive");
  if (!(opts->rs_sigma >= 0.0f)) return fail(NEDF_ERR_SHAPE, "rs_sigma must be >= 0");
  if (opts->rs_sigma > 0.0f && !(opts->rs_samples == 8 || opts->rs_samples == 16 || opts->rs_samples == 32))
    return fail(NEDF_ERR_SHAPE, "rs_samples must be 8, 16 or 32");
  Prepared P;
  int32_t st = prepare_scene(scene, opts->dtype, P);
  if (st) return st;
  for (int i = 0; i < scene->n_objects; ++i)
    if (((P.mlp >> i) & 1u) && !shade_supported(opts->dtype, scene->objects[i].density.shape))
      return fail(NEDF_ERR_UNSUPPORTED, "shading needs NeRF objects with a colour branch (256x8, L10, rgb 128, dir L4)");
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!depth || !id || !rgb) return fail(NEDF_ERR_NULL, "depth, id and rgb are required");
  if (!aligned16(depth) || !aligned16(id) || !aligned16(rgb)) return fail(NEDF_ERR_ALIGN, "buffers must be 16-byte aligned");
  WsLayout lay;
  st = prepare_ws(P, rs, 0, ws, ws_bytes, lay);
  if (st) return st;
  set_rays(P.k, rs);
  KArgs& k = P.k;
  k.depth = const_cast<float*>(depth);
  k.rgb = rgb;
  k.shade_K = K;
  k.shade_h = opts->h;
  k.rs_sigma = opts->rs_sigma;
  k.shade_chord = 0;
  for (int c = 0; c < 3; ++c) k.clear_rgb[c] = opts->clear_rgb[c];
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, k.status);
  stage_shade(k, s, id, P.nerf, opts->dtype, opts->rs_sigma > 0.0f ? opts->rs_samples : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "nedf_shade_deferred");
  return NEDF_OK;
}

extern "C" int32_t nedf_shadow(const nedf_scene* scene, const nedf_rays* rays, const float* depth, const int32_t* id,
                               const float* lights, int32_t n_lights, const nedf_shadow_opts* opts, float* shadow,
                               float* rgb_inout, void* ws, size_t ws_bytes, nedf_stream_t stream) {
  if (!opts) return fail(NEDF_ERR_NULL, "shadow opts are NULL");
  if (n_lights < 0 || n_lights > 8) return fail(NEDF_ERR_SHAPE, "n_lights must be 0..8");
  if (n_lights > 0 && !lights) return fail(NEDF_ERR_NULL, "lights is NULL");
  if (!(opts->beta > 0.0f && opts->beta < 1.0f)) return fail(NEDF_ERR_SHAPE, "beta must be in (0, 1)");
  if (!(opts->eps >= 0.0f)) return fail(NEDF_ERR_SHAPE, "eps must be >= 0");
  if (opts->method != 0 && opts->method != 1) return fail(NEDF_ERR_SHAPE, "method must be 0 (NeDF) or 1 (marcher)");
  if (n_lights < 32 && (opts->directional_mask >> n_lights) != 0)
    return fail(NEDF_ERR_SHAPE, "directional_mask names a light beyond n_lights");
  if (opts->directional_mask && !(opts->dir_distance > 0.0f))
    return fail(NEDF_ERR_SHAPE, "directional lights need dir_distance > 0");
  int32_t st = opts->method == 0 ? check_infer_opts(&opts->infer) : check_march_opts(&opts->infer.march);
  if (st) return st;
  const int32_t dtype = opts->method == 0 ? opts->infer.dtype : opts->infer.march.dtype;
  Prepared P;
  st = prepare_scene(scene, dtype, P);
  if (st) return st;
  if (opts->method == 0 && (P.mlp & ~P.nedf)) return fail(NEDF_ERR_UNSUPPORTED, "NeDF shadows need an intersection network on every MLP object");
  RaySrcHost rs;
  st = check_rays(rays, rs);
  if (st) return st;
  if (rs.n == 0) return NEDF_OK;
  if (!depth || !id || !shadow) return fail(NEDF_ERR_NULL, "depth, id and shadow are required");
  if (!aligned16(depth) || !aligned16(id) || !aligned16(shadow) || (rgb_inout && !aligned16(rgb_inout)))
    return fail(NEDF_ERR_ALIGN, "buffers must be 16-byte aligned");
  const size_t extra = size_t(rs.n) * SHADOW_EXTRA_PER_RAY;
  WsLayout lay;
  st = prepare_ws(P, rs, extra, ws, ws_bytes, lay);
  if (st) return st;
  uint8_t* w = static_cast<uint8_t*>(ws);
  float* so = reinterpret_cast<float*>(w + lay.extra);
  float* sd = so + 3 * rs.n;
  float* dist = sd + 3 * rs.n;
  float* depth_l = dist + rs.n;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // primary-ray view of the scene (for x = o + D d)
  Prepared Pp = P;
  set_rays(Pp.k, rs);
  Pp.k.depth = const_cast<float*>(depth);
  stage_shadow_init(Pp.k, s, shadow);
  // shadow-ray view: explicit rays from the workspace
  RaySrcHost sr;
  std::memset(&sr, 0, sizeof(sr));
  sr.kind = 1;
  sr.o = so;
  sr.d = sd;
  sr.n = rs.n;
  Prepared Ps = P;
  set_rays(Ps.k, sr);
  Ps.k.depth = depth_l;
  Ps.k.id = nullptr;
  Ps.k.opacity = nullptr;
  // one shadow ray per pixel: cull the array in image tiles
  Ps.k.ray_grid_w = rs.kind == 0 ? rs.width : 0;
  prof_mark("shadow", s, true);
  for (int m = 0; m < n_lights; ++m) {
    const bool dirl = (opts->directional_mask >> m) & 1u;
    float Lm[3] = {lights[3 * m], lights[3 * m + 1], lights[3 * m + 2]};
    if (dirl) {
      const float nrm = std::sqrt(Lm[0] * Lm[0] + Lm[1] * Lm[1] + Lm[2] * Lm[2]);
      if (!(nrm > 0.0f)) return fail(NEDF_ERR_SHAPE, "a directional light needs a nonzero direction");
      for (float& v : Lm) v /= nrm;
    }
    stage_shadow_rays(Pp.k, s, id, Lm, dirl ? opts->dir_distance : 0.0f, so, sd, dist);
    if (opts->method == 0) {
      apply_march_opts(Ps.k, opts->infer.march);
      nedf_infer_opts io = opts->infer;
      io.refine_steps = 0;  // the occlusion test needs no refined depth
      // only whether a hit lies closer than |L - x| - eps matters: pairs that
      // cannot change that are skipped (the depth buffer of the shadow rays is
      // then exact below that distance only)
      Ps.k.ray_tmax = dist;
      Ps.k.tmax_eps = opts->eps;
      run_infer(Ps, dtype, io, s);
      Ps.k.ray_tmax = nullptr;
    } else {
      apply_march_opts(Ps.k, opts->infer.march);
      Ps.k.clip = 1;
      run_march(Ps, dtype, s);
    }
    stage_shadow_apply(Pp.k, s, id, depth_l, dist, opts->eps, opts->beta, shadow);
  }
  if (rgb_inout) stage_composite(Pp.k, s, shadow, rgb_inout);
  prof_mark("shadow", s, false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "nedf_shadow");
  return NEDF_OK;
}

extern "C" int32_t nedf_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  g_prof_open.clear();
  g_prof_on = on != 0;
  return NEDF_OK;
}

extern "C" int32_t nedf_profile_read(int32_t max_stages, char* names, double* total_ms, int32_t* counts,
                                     int32_t* n_stages) {
  if (!names || !total_ms || !counts || !n_stages) return fail(NEDF_ERR_NULL, "nedf_profile_read: NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<std::string> order;
  std::map<std::string, std::pair<double, int>> agg;
  for (auto& r : g_prof_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(NEDF_ERR_HIP, "nedf_profile_read: event sync failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    std::string n(r.name);
    if (!agg.count(n)) order.push_back(n);
    agg[n].first += ms;
    agg[n].second += 1;
  }
  int32_t k = 0;
  for (auto& n : order) {
    if (k >= max_stages) break;
    std::strncpy(names + 64 * k, n.c_str(), 63);
    names[64 * k + 63] = 0;
    total_ms[k] = agg[n].first;
    counts[k] = agg[n].second;
    ++k;
  }
  *n_stages = k;
  return NEDF_OK;
}


namespace {
int32_t check_train_shape(const nedf_mlp_shape* s) {
  if (!s) return fail(NEDF_ERR_NULL, "shape is NULL");
  if (s->in_kind == NEDF_IN_POINTS16) {
    if (s->width != 256 || s->enc_L != 10 || s->rgb_width != 0 || s->n_out != 1 + NEDF_CLS_COARSE + NEDF_CLS_FINE)
      return fail(NEDF_ERR_UNSUPPORTED, "classifier training needs width 256, L10, 193 outputs");
    if (s->n_hidden < 1 || 2 * s->n_hidden + 2 > NEDF_TRAIN_MAX_LAYERS)
      return fail(NEDF_ERR_SHAPE, "classifier training takes 1..16 residual blocks");
    return NEDF_OK;
  }
  if (s->width != 256 || s->n_out != 2 || s->rgb_width != 0) return fail(NEDF_ERR_UNSUPPORTED, "training needs width 256, n_out 2, no colour branch");
  if (s->n_hidden < 1 || s->n_hidden > NEDF_MAX_LAYERS) return fail(NEDF_ERR_SHAPE, "n_hidden must be 1..16");
  if (s->in_kind != NEDF_IN_PLUECKER && s->in_kind != NEDF_IN_XYZ) return fail(NEDF_ERR_SHAPE, "bad in_kind");
  if (s->enc_L < 0 || s->enc_L > 12) return fail(NEDF_ERR_SHAPE, "enc_L must be 0..12");
  return NEDF_OK;
}
}  // namespace

extern "C" size_t nedf_train_state_bytes(const nedf_mlp_shape* shape) {
  if (check_train_shape(shape)) return 0;
  return nedf_train_layout_of(*shape).total;
}

extern "C" size_t nedf_train_workspace_size(const nedf_mlp_shape* shape, int32_t B) {
  if (check_train_shape(shape) || B <= 0) return 0;
  return train_ws_bytes(*shape, B);
}

extern "C" int32_t nedf_train_init(const nedf_mlp_shape* shape, const float* const* W, const float* const* b,
                                   void* state, size_t state_bytes, nedf_stream_t stream) {
  int32_t st = check_train_shape(shape);
  if (st) return st;
  if (!W || !b || !state) return fail(NEDF_ERR_NULL, "nedf_train_init: NULL argument");
  const nedf_train_layout tl = nedf_train_layout_of(*shape);
  if (state_bytes < tl.total) return fail(NEDF_ERR_WORKSPACE, "nedf_train_init: state buffer too small");
  if (!aligned16(state)) return fail(NEDF_ERR_ALIGN, "state must be 16-byte aligned");
  for (int i = 0; i < tl.n_layers; ++i)
    if (!W[i] || !b[i]) return fail(NEDF_ERR_NULL, "nedf_train_init: NULL layer pointer");
  hipError_t e = launch_train_init(*shape, W, b, static_cast<uint8_t*>(state), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_train_init");
  return NEDF_OK;
}

extern "C" int32_t nedf_train_step(const nedf_mlp_shape* shape, void* state, const float* o_l, const float* d_l,
                                   const float* depth_label, const uint8_t* hit_label, int32_t B,
                                   const nedf_train_opts* opts, float* loss_out, void* ws, size_t ws_bytes,
                                   nedf_stream_t stream) {
  int32_t st = check_train_shape(shape);
  if (st) return st;
  if (!state || !o_l || !d_l || !depth_label || !hit_label || !opts || !loss_out || !ws)
    return fail(NEDF_ERR_NULL, "nedf_train_step: NULL argument");
  if (B <= 0 || B % 256 != 0) return fail(NEDF_ERR_SHAPE, "batch must be a positive multiple of 256");
  if (!aligned16(state) || !aligned16(o_l) || !aligned16(d_l) || !aligned16(depth_label) || !aligned16(ws))
    return fail(NEDF_ERR_ALIGN, "nedf_train_step: misaligned pointer");
  if (ws_bytes < train_ws_bytes(*shape, B)) return fail(NEDF_ERR_WORKSPACE, "workspace smaller than nedf_train_workspace_size()");
  if (!(opts->lr >= 0.0f) || !(opts->beta1 >= 0.0f && opts->beta1 < 1.0f) || !(opts->beta2 >= 0.0f && opts->beta2 < 1.0f) ||
      !(opts->eps > 0.0f) || !(opts->bound > 0.0f))
    return fail(NEDF_ERR_SHAPE, "bad Adam / loss options");
  hipError_t e = launch_train_step(*shape, static_cast<uint8_t*>(state), o_l, d_l, depth_label, hit_label, B,
                                   opts->lr, opts->beta1, opts->beta2, opts->eps, opts->w_hit, opts->bound, loss_out,
                                   static_cast<uint8_t*>(ws), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_train_step");
  return NEDF_OK;
}

extern "C" int32_t nedf_train_export(const nedf_mlp_shape* shape, const void* state, int32_t which, float* const* W,
                                     float* const* b, nedf_stream_t stream) {
  int32_t st = check_train_shape(shape);
  if (st) return st;
  if (!state || !W || !b) return fail(NEDF_ERR_NULL, "nedf_train_export: NULL argument");
  if (which != 0 && which != 1) return fail(NEDF_ERR_SHAPE, "which must be 0 (weights) or 1 (gradients)");
  const nedf_train_layout tl = nedf_train_layout_of(*shape);
  for (int i = 0; i < tl.n_layers; ++i)
    if (!W[i] || !b[i]) return fail(NEDF_ERR_NULL, "nedf_train_export: NULL layer pointer");
  hipError_t e = launch_train_export(*shape, static_cast<const uint8_t*>(state), W, b, which == 1,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_train_export");
  return NEDF_OK;
}

extern "C" size_t nedf_fp8_calibrate_workspace_size(const nedf_mlp_shape* shape, int32_t B) {
  if (check_train_shape(shape) || B <= 0) return 0;
  if (shape->in_kind == NEDF_IN_POINTS16) {
    set_error("FP8 calibration covers the regression-form network");
    return 0;
  }
  return fp8_calibrate_ws_bytes(*shape, B);
}

extern "C" int32_t nedf_fp8_calibrate(const nedf_mlp_shape* shape, const float* const* W, const float* const* b,
                                      const float* o_l, const float* d_l, int32_t B, float* scales, void* ws,
                                      size_t ws_bytes, nedf_stream_t stream) {
  int32_t st = check_train_shape(shape);
  if (st) return st;
  if (shape->in_kind == NEDF_IN_POINTS16)
    return fail(NEDF_ERR_UNSUPPORTED, "nedf_fp8_calibrate: FP8 calibration covers the regression-form network");
  if (!W || !b || !o_l || !d_l || !scales || !ws) return fail(NEDF_ERR_NULL, "nedf_fp8_calibrate: NULL argument");
  if (B <= 0 || B % 256 != 0) return fail(NEDF_ERR_SHAPE, "calibration batch must be a positive multiple of 256");
  if (!aligned16(ws) || !aligned16(o_l) || !aligned16(d_l)) return fail(NEDF_ERR_ALIGN, "nedf_fp8_calibrate: misaligned pointer");
  if (ws_bytes < fp8_calibrate_ws_bytes(*shape, B)) return fail(NEDF_ERR_WORKSPACE, "workspace smaller than nedf_fp8_calibrate_workspace_size()");
  hipError_t e = launch_fp8_calibrate(*shape, W, b, o_l, d_l, B, scales, static_cast<uint8_t*>(ws),
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_fp8_calibrate");
  return NEDF_OK;
}


// ---- tuning table and autotuner ---------------------------------------------
namespace {
std::mutex g_tune_mu;
// [kernel][dtype]: 10 * workgroups per CU + chunks per superchunk; for
// NEDF_TUNE_SLABS the number of depth slabs of the network stage
int g_tune[3][3] = {{11, 1012, 14}, {11, 1012, 14}, {8, 8, 8}};

int tune_candidates(int kernel, int dtype, int32_t* out) {
  if (kernel < 0 || kernel > 2 || dtype < 0 || dtype > 2) return 0;
  if (kernel == NEDF_TUNE_SLABS) {
    for (int i = 0; i < 6; ++i) out[i] = 1 << i;
    return 6;
  }
  if (dtype == NEDF_F32) { out[0] = 11; return 1; }
  if (dtype == NEDF_BF16) {
    out[0] = 11; out[1] = 12; out[2] = 21; out[3] = 111; out[4] = 112; out[5] = 1011; out[6] = 1012;
    return 7;
  }
  if (kernel == NEDF_TUNE_NEDF) {
    out[0] = 11; out[1] = 12; out[2] = 14; out[3] = 21; out[4] = 22; out[5] = 1011; out[6] = 1012; out[7] = 1014;
    return 8;
  }
  return 0;  // no FP8 marcher
}
}  // namespace

namespace nedf {
int tune_value(int kernel, int dtype) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (kernel < 0 || kernel > 2 || dtype < 0 || dtype > 2) return 1;
  return g_tune[kernel][dtype];
}
}  // namespace nedf

extern "C" int32_t nedf_tune_candidates(int32_t kernel, int32_t dtype, int32_t* out, int32_t* n) {
  if (!out || !n) return fail(NEDF_ERR_NULL, "nedf_tune_candidates: NULL argument");
  *n = tune_candidates(kernel, dtype, out);
  if (*n == 0) return fail(NEDF_ERR_UNSUPPORTED, "no tunable kernel for this (kernel, dtype)");
  return NEDF_OK;
}

extern "C" int32_t nedf_tune_get(int32_t kernel, int32_t dtype, int32_t* value) {
  if (!value) return fail(NEDF_ERR_NULL, "nedf_tune_get: NULL argument");
  int32_t c[NEDF_TUNE_MAX];
  if (tune_candidates(kernel, dtype, c) == 0) return fail(NEDF_ERR_UNSUPPORTED, "no tunable kernel for this (kernel, dtype)");
  *value = tune_value(kernel, dtype);
  return NEDF_OK;
}

extern "C" int32_t nedf_tune_set(int32_t kernel, int32_t dtype, int32_t value) {
  int32_t c[NEDF_TUNE_MAX];
  const int n = tune_candidates(kernel, dtype, c);
  if (n == 0) return fail(NEDF_ERR_UNSUPPORTED, "no tunable kernel for this (kernel, dtype)");
  bool ok = false;
  for (int i = 0; i < n; ++i) ok |= c[i] == value;
  if (!ok) return fail(NEDF_ERR_UNSUPPORTED, "value is not an instantiated candidate");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[kernel][dtype] = value;
  return NEDF_OK;
}

extern "C" int32_t nedf_autotune(int32_t kernel, int32_t dtype, const nedf_scene* scene, const nedf_rays* rays,
                                 const void* opts, float* depth, int32_t* id, void* ws, size_t ws_bytes,
                                 int32_t reps, nedf_stream_t stream, nedf_tune_report* report) {
  if (!scene || !rays || !opts || !report) return fail(NEDF_ERR_NULL, "nedf_autotune: NULL argument");
  if (reps < 1 || reps > 100) return fail(NEDF_ERR_SHAPE, "reps must be 1..100");
  int32_t cand[NEDF_TUNE_MAX];
  const int n = tune_candidates(kernel, dtype, cand);
  if (n == 0) return fail(NEDF_ERR_UNSUPPORTED, "no tunable kernel for this (kernel, dtype)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto run = [&]() -> int32_t {
    if (kernel == NEDF_TUNE_MARCH)
      return nedf_march_depth(scene, rays, static_cast<const nedf_march_opts*>(opts), depth, id, nullptr, ws,
                              ws_bytes, stream);
    return nedf_infer_depth_id(scene, rays, static_cast<const nedf_infer_opts*>(opts), depth, id, ws, ws_bytes,
                               stream);
  };
  const int32_t saved = tune_value(kernel, dtype);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(NEDF_ERR_HIP, "nedf_autotune: event creation failed");
  }
  int32_t st = NEDF_OK;
  int best = -1;
  std::memset(report, 0, sizeof(*report));
  report->kernel = kernel;
  report->dtype = dtype;
  report->n_candidates = n;
  for (int i = 0; i < n && st == NEDF_OK; ++i) {
    report->candidate[i] = cand[i];
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[kernel][dtype] = cand[i];
    }
    st = run();  // warm-up
    if (st) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == NEDF_OK; ++r) st = run();
    (void)hipEventRecord(e1, s);
    if (st) break;
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(NEDF_ERR_HIP, "nedf_autotune: event sync failed"); break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    report->ms[i] = ms / float(reps);
    if (best < 0 || report->ms[i] < report->ms[best]) best = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (st != NEDF_OK || best < 0) {
    g_tune[kernel][dtype] = saved;
    return st ? st : fail(NEDF_ERR_HIP, "nedf_autotune: no candidate ran");
  }
  g_tune[kernel][dtype] = cand[best];
  report->chosen = cand[best];
  return NEDF_OK;
}
